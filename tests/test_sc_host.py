"""The library's sparse-grid construction (host code, no GPU needed) against
the oracle (Sec. 4.1.2, global SC methods), and host-side argument checks of
the collocation entry points.

The two sides compute the Clenshaw-Curtis weights differently (the library
from the explicit cosine-sum formula, the oracle by integrating the Lagrange
basis with a Gauss-Legendre rule) and add the combination terms in different
orders, so weights agree to rounding: the terms carry binomial coefficients
up to binom(15, 4) = 1365 at d = 16, hence atol 1e-11.  Digits agree bit for
bit."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import sc

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1607_00693_amd",
                   "libstomsfem.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem
    stomsfem.lib()
    return stomsfem


@pytest.mark.parametrize("d,level", [(1, 0), (1, 5), (2, 4), (3, 3), (5, 2), (16, 1), (16, 2), (16, 3), (4, 6)])
def test_sparse_grid_matches_the_oracle(sm, d, level):
    dg, w = sm.sparse_grid(d, level)
    dr, wr = sc.sparse_grid(d, level)
    assert dg.shape == dr.shape
    assert (dg == dr).all()
    np.testing.assert_allclose(w, wr, rtol=0, atol=1e-11)
    assert abs(w.sum() - 1.0) < 1e-10


def test_sparse_grid_argument_checks(sm):
    n = C.c_int64(-5)
    L = sm.lib()
    assert L.stomsfem_sparse_grid(0, 2, 0, C.byref(n), None, None) == sm.EINVAL and n.value == 0
    assert L.stomsfem_sparse_grid(3, 9, 0, C.byref(n), None, None) == sm.EINVAL
    assert L.stomsfem_sparse_grid(3, -1, 0, C.byref(n), None, None) == sm.EINVAL
    assert L.stomsfem_sparse_grid(3, 2, 0, None, None, None) == sm.EINVAL
    # more than 2e6 combination terms
    assert L.stomsfem_sparse_grid(200, 8, 0, C.byref(n), None, None) == sm.EINVAL
    # count only, then a buffer one row short
    assert L.stomsfem_sparse_grid(3, 2, 0, C.byref(n), None, None) == 0 and n.value == 25
    w = np.zeros(24)
    assert L.stomsfem_sparse_grid(3, 2, 24, C.byref(n), None, w.ctypes.data_as(C.c_void_p)) == sm.EINVAL
    assert n.value == 25


def test_collocation_entry_argument_checks(sm):
    L = sm.lib()
    fam = sm.BumpFamily(4, 0.25, 1 / 32, 2.0, 1.8, 0.5)
    lv = np.full((4, 4), -1, dtype=np.int32)
    lv[:, 0] = 0
    dg = np.zeros((3, 16), dtype=np.int32)
    h = C.c_void_p()
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    args = lambda **kw: dict(dict(ncx=2, ncy=2, m=8, level=2, lo=-1.0, hi=1.0, n=3, lvp=P(lv), dgp=P(dg)), **kw)

    def build(**kw):
        a = args(**kw)
        return L.stomsfem_sc_build(a["ncx"], a["ncy"], a["m"], a["lvp"], C.byref(fam), a["level"], a["lo"], a["hi"],
                                   a["dgp"], a["n"], C.byref(h), None)
    assert build(level=9) == sm.EINVAL
    assert build(n=0) == sm.EINVAL
    assert build(lo=1.0) == sm.EINVAL
    assert build(m=49) == sm.EINVAL
    assert build(dgp=None) == sm.EINVAL
    bad = dg.copy()
    bad[1, 3] = 5  # digits of level 2 are 0..4
    assert build(dgp=P(bad)) == sm.EINVAL
    lv2 = lv.copy()
    lv2[0, :2] = [3, 1]  # not increasing
    assert build(lvp=P(lv2)) == sm.EINVAL
    assert L.stomsfem_sc_apply(None, None, 16, 1, None, None, None) == sm.EINVAL
    assert L.stomsfem_quadrature(None, None, 0, 4, None, None, None) == sm.EINVAL
    assert L.stomsfem_quadrature(None, None, 4, 0, None, None, None) == sm.EINVAL
