"""Pins of the random-interpolation oracle (Sec. 3.1, Algorithms 1-2,
Thm. 3.3) against closed forms, library routines and the plain path."""
import itertools

import numpy as np
import pytest

from oracle import core, ri
from paper_1607_00693_amd import workloads as W


def test_cgl_nodes_closed_forms():
    np.testing.assert_allclose(ri.cgl_nodes(2), [1.0, -1.0], atol=0)
    np.testing.assert_allclose(ri.cgl_nodes(3), [1.0, 0.0, -1.0], atol=1e-16)
    h = np.sqrt(0.5)
    np.testing.assert_allclose(ri.cgl_nodes(5), [1.0, h, 0.0, -h, -1.0], atol=1e-15)
    # affine map to a box keeps the end points and the Chebyshev spacing
    t = ri.cgl_nodes(5, -3.0, 1.0)
    np.testing.assert_allclose(t, [1.0, -1.0 + 2 * h, -1.0, -1.0 - 2 * h, -3.0], atol=1e-15)
    # extrema of the Chebyshev polynomial T_nu: |T_nu(t_j)| = 1 with alternating sign
    for nn in (4, 7, 9):
        t = ri.cgl_nodes(nn)
        Tn = np.polynomial.chebyshev.chebval(t, [0] * (nn - 1) + [1])
        np.testing.assert_allclose(Tn, (-1.0) ** np.arange(nn), atol=1e-13)


def test_lagrange_basis_kronecker_and_partition_of_unity():
    for nn in (2, 5, 8):
        t = ri.cgl_nodes(nn, -0.7, 2.0)
        np.testing.assert_allclose(ri.lagrange_basis(t, t), np.eye(nn), atol=1e-13)
        x = W.uniform_array(50, -0.7, 2.0, seed=5)
        B = ri.lagrange_basis(x, t)
        np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-13)
        # reproduces the identity function (degree 1 <= nu)
        np.testing.assert_allclose(B @ t, x, atol=1e-13)


def test_one_variable_matches_polyfit():
    # one local variable: the interpolant is the unique polynomial of degree
    # nu through the node values, which numpy's least-squares fit of that
    # degree also is
    nn = 6
    t = ri.cgl_nodes(nn)
    vals = W.uniform_array((nn, 10), -1, 1, seed=11)
    x = W.uniform_array((40, 1), -1, 1, seed=12)
    got = ri.ri_eval(vals, t, x)
    for e in range(10):
        c = np.polyfit(t, vals[:, e], nn - 1)
        np.testing.assert_allclose(got[:, e], np.polyval(c, x[:, 0]), atol=1e-11)


@pytest.mark.parametrize("k,nn", [(2, 4), (3, 3), (4, 3)])
def test_tensor_polynomial_exactness(k, nn):
    # exact for every polynomial of degree <= nu in each variable (Thm. 3.3 has
    # no error term then); one degree more is not reproduced
    t = ri.cgl_nodes(nn, -2.0, 1.0)
    coef = W.uniform_array((10, k, nn + 1), -1, 1, seed=20 + k)
    x = W.uniform_array((25, k), -2.0, 1.0, seed=30 + k)

    def q(pts, deg):
        out = np.ones((len(pts), 10))
        for e in range(10):
            for i in range(k):
                out[:, e] *= np.polyval(coef[e, i, -(deg + 1):], pts[:, i])
        return out

    grid = np.array(list(itertools.product(t, repeat=k)))  # variable 0 slowest
    np.testing.assert_allclose(ri.ri_eval(q(grid, nn - 1), t, x), q(x, nn - 1), atol=1e-11)
    miss = np.abs(ri.ri_eval(q(grid, nn), t, x) - q(x, nn)).max()
    assert miss > 1e-4


def _mesh8():
    wl = W.MESH8
    fam = wl.coef_params()
    lv = ri.local_vars_bumps(wl.nc, wl.m, wl.g, wl.rho)
    return wl, fam, lv


def test_local_vars_mesh8_counts():
    wl, fam, lv = _mesh8()
    assert np.bincount([len(v) for v in lv]).tolist() == [0, 4, 24, 0, 36]
    # corner patch 0 sees bump 0 only; an interior patch sees the 2 x 2 bumps around it
    assert lv[0] == [0]
    assert lv[9] == [0, 1, 4, 5]


def test_nodes_reproduce_plain_solve_with_nonlocal_variables_free():
    # at a tensor node the interpolant returns the plain S of the full problem,
    # whatever the variables that are not local to the patch are
    wl, fam, lv = _mesh8()
    nn = 4
    mod = ri.ri_offline(wl.nc, wl.m, fam, lv, nn, -1.0, 1.0, patches=[9, 1])
    nodes = ri.cgl_nodes(nn)
    for K, digits in ((9, (1, 3, 0, 2)), (1, (2, 0))):
        xi = W.uniform_xi(3, wl.nxi, seed=40 + K)
        for i, j in enumerate(lv[K]):
            xi[:, j] = nodes[digits[i]]
        a = core.coef_bumps(xi, wl.nfine, **fam)
        S_full, _, _ = core.upscale(a, wl.nc, wl.nc, wl.m)
        got = ri.ri_eval(mod["tables"][K], nodes, xi[:, lv[K]])
        sc = np.abs(S_full[:, K]).max()
        np.testing.assert_allclose(got, S_full[:, K], atol=1e-12 * sc)
        c = sum(d * nn ** (len(digits) - 1 - i) for i, d in enumerate(digits))
        np.testing.assert_allclose(mod["tables"][K][c], S_full[0, K], atol=1e-12 * sc)


def test_exponential_convergence_in_nodes():
    # Thm. 3.3: the error decays exponentially in nu for a coefficient analytic
    # in xi; measured: 3e-3, 7e-6, 7e-9 at 3, 5, 7 nodes per variable
    wl, fam, lv = _mesh8()
    xi = W.uniform_xi(8, wl.nxi, seed=50)
    for K in (1, 9):
        Sp = ri.patch_S(xi, K, wl.nc, wl.m, fam)
        errs = []
        for nn in (3, 5, 7):
            mod = ri.ri_offline(wl.nc, wl.m, fam, lv, nn, -1.0, 1.0, patches=[K])
            errs.append(np.abs(ri.ri_eval(mod["tables"][K], mod["nodes"], xi[:, lv[K]]) - Sp).max()
                        / np.abs(Sp).max())
        assert errs[0] < 1e-2 and errs[1] < 3e-5 and errs[2] < 3e-8
        assert errs[1] < 1e-2 * errs[0] and errs[2] < 1e-2 * errs[1]


def test_out_of_box_pairs_are_solved_plainly():
    wl, fam, lv = _mesh8()
    sub = [0, 1, 9]
    mod = ri.ri_offline(wl.nc, wl.m, fam, lv, 5, -0.6, 0.6, patches=sub)
    xi = W.uniform_xi(12, wl.nxi, seed=60)
    # restrict the oracle's online stage to the patches that have tables
    M = wl.M
    mod_all = dict(mod, tables={K: mod["tables"].get(K, np.zeros((5 ** len(lv[K]), 10))) for K in range(M)})
    S, fb = ri.ri_online(mod_all, xi, wl.nc, wl.m, fam)
    a = core.coef_bumps(xi, wl.nfine, **fam)
    Sp, _, _ = core.upscale(a, wl.nc, wl.nc, wl.m)
    for K in sub:
        out = np.any(np.abs(xi[:, lv[K]]) > 0.6, axis=1)
        np.testing.assert_array_equal(fb[:, K], out)
        assert out.any() and (~out).any()
        sc = np.abs(Sp[:, K]).max()
        np.testing.assert_allclose(S[out, K], Sp[out, K], atol=1e-13 * sc)
        # inside the box the interpolant is accurate to the 5-node level
        assert np.abs(S[~out, K] - Sp[~out, K]).max() < 1e-5 * sc
