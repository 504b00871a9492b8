"""Pins of the oracle's sparse-grid stochastic collocation with
search-and-plug-in dictionaries (Sec. 3.3, global SC methods; Sec. 5.1, the
second experiment) against facts fixed outside it: the classical
Clenshaw-Curtis weights, hand-derived small grids (tests/golden), the point
counts that follow from the numbers of new points per nested level, exact
integration of polynomials of total degree <= 2L + 1 (Novak and Ritter), the
plain path at every collocation point, and a Monte Carlo estimate of the
same expectation."""
import os

import numpy as np
import pytest

from oracle import sc
from paper_1607_00693_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sparse_grid_cc_d2.txt")


def test_one_dimensional_clenshaw_curtis_weights():
    # n = 3: Simpson's rule; n = 5: 1/15, 8/15, 4/5, 8/15, 1/15 for int dx
    # (halved for the probability measure); n = 9: symmetric, positive, exact
    # for degree 9 but not for the Gauss-Legendre-exact degree 10 moment
    t, w = sc.cc_rule(2)
    np.testing.assert_allclose(t, [1, 0, -1], atol=1e-16)
    np.testing.assert_allclose(w, [1 / 6, 2 / 3, 1 / 6], rtol=1e-14)
    _, w = sc.cc_rule(3)
    np.testing.assert_allclose(w, np.array([1, 8, 12, 8, 1]) / 30, rtol=1e-14)
    t, w = sc.cc_rule(4)
    assert (w > 0).all() and np.allclose(w, w[::-1], rtol=1e-13)
    for k in range(10):
        assert abs(w @ t**k - (1 / (k + 1) if k % 2 == 0 else 0)) < 1e-14
    assert abs(w @ t**10 - 1 / 11) > 1e-6


def _golden():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    out = {}
    for lv, c0, c1, num, den in rows:
        out.setdefault(int(lv), {})[(int(c0), int(c1))] = int(num) / int(den)
    return out


@pytest.mark.parametrize("level", [1, 2])
def test_hand_derived_grids(level):
    ref = _golden()[level]
    D, w = sc.sparse_grid(2, level)
    assert [tuple(r) for r in D] == sorted(ref)
    np.testing.assert_allclose(w, [ref[tuple(r)] for r in D], rtol=0, atol=1e-15)


def _count(d, level):
    # points of the nested grid = sum over |i| - d <= level of the products of
    # the numbers of points new at each level: 1, 2, 2, 4, 8, ...
    new = [0, 1, 2] + [2 ** (i - 2) for i in range(3, 12)]
    import itertools
    tot = 0
    for idx in itertools.product(range(1, level + 2), repeat=d):
        if sum(idx) - d <= level:
            tot += int(np.prod([new[i] for i in idx]))
    return tot


@pytest.mark.parametrize("d,level", [(1, 3), (2, 4), (3, 3), (4, 2), (5, 2)])
def test_point_counts(d, level):
    D, w = sc.sparse_grid(d, level)
    assert len(w) == _count(d, level)
    assert len({tuple(r) for r in D}) == len(w)


def test_known_counts_two_and_three_dimensions():
    assert [len(sc.sparse_grid(2, L)[1]) for L in range(5)] == [1, 5, 13, 29, 65]
    assert [len(sc.sparse_grid(3, L)[1]) for L in range(5)] == [1, 7, 25, 69, 177]


@pytest.mark.parametrize("d,level", [(2, 1), (2, 3), (3, 2), (4, 2), (3, 3)])
def test_polynomial_exactness(d, level):
    # exact for every monomial of total degree <= 2 level + 1
    import itertools
    D, w = sc.sparse_grid(d, level)
    X = sc.node_values(D, level)
    for a in itertools.product(range(2 * level + 2), repeat=d):
        if sum(a) > 2 * level + 1:
            continue
        exact = np.prod([1 / (k + 1) if k % 2 == 0 else 0.0 for k in a])
        got = w @ np.prod(X ** np.array(a), axis=1)
        assert abs(got - exact) < 1e-13, (a, got, exact)


def test_one_dimension_is_the_clenshaw_curtis_rule():
    for L in range(5):
        D, w = sc.sparse_grid(1, L)
        t, w1 = sc.cc_rule(L + 1)
        np.testing.assert_allclose(sc.node_values(D[:, 0], L), t, atol=1e-15)
        np.testing.assert_allclose(w, w1, rtol=1e-14)


def _fam():
    return W.MESH8.coef_params()


def test_dictionary_plug_in_equals_the_plain_path():
    # locality: S_K at a collocation point is the dictionary entry of its
    # local point, to rounding (in fact bit for bit)
    from oracle import ri
    wl = W.MESH8
    fam = _fam()
    lv = ri.local_vars_bumps(wl.nc, wl.m, fam["g"], fam["rho"])
    D, _ = sc.sparse_grid(wl.nxi, 2)
    model = sc.sc_offline(wl.nc, wl.m, fam, lv, D, 2)
    assert sum(len(model["dicts"][K][0]) for K in range(wl.M)) < len(D) * wl.M / 4
    S = sc.sc_plug_in(model, D)
    S_ref = sc.sc_direct(wl.nc, wl.m, fam, D, 2)
    assert np.abs(S - S_ref).max() <= 1e-13 * np.abs(S_ref).max()


def test_collocation_converges_to_the_expectation():
    # E[u_H] by sparse-grid collocation at levels 1..3 against level 4, and
    # level 4 against a Monte Carlo estimate with its standard error
    from oracle import core, ri
    wl = W.MESH8
    fam = _fam()
    lv = ri.local_vars_bumps(wl.nc, wl.m, fam["g"], fam["rho"])
    D4, w4 = sc.sparse_grid(wl.nxi, 4)
    model = sc.sc_offline(wl.nc, wl.m, fam, lv, D4, 4)
    means = {}
    for L in (1, 2, 3, 4):
        D, w = sc.sparse_grid(wl.nxi, L)
        D4scaled = D * (2 ** 4 // sc.digit_base(L))  # same nodes on the level-4 digit grid
        U, _, _ = core.coarse_solve(sc.sc_plug_in(model, D4scaled), wl.nc, wl.nc)
        means[L] = sc.quadrature(U, w)[0]
    err = [np.linalg.norm(means[L] - means[4]) for L in (1, 2, 3)]
    assert err[0] > err[1] > err[2], err
    N = 16000
    xi = W.uniform_xi(N, wl.nxi, 9001)
    a = core.coef_bumps(xi, wl.nfine, **fam)
    S, st, _ = core.upscale(a, wl.nc, wl.nc, wl.m)
    U, _, _ = core.coarse_solve(S, wl.nc, wl.nc)
    se = U.std(axis=0) / np.sqrt(N)
    assert np.all(np.abs(U.mean(axis=0) - means[4]) < 4.5 * se)
    assert err[2] < 0.1 * se.max()
