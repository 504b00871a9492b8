"""Pins of the oracle's sparse-grid stochastic collocation with
search-and-plug-in dictionaries (Sec. 4.1.2, global SC methods; the
collocation experiment of Sec. 5.2) against facts fixed outside it: the classical
Clenshaw-Curtis weights, hand-derived small grids (tests/golden), the point
counts that follow from the numbers of new points per nested level, exact
integration of polynomials of total degree <= 2L + 1 (Novak and Ritter), the
plain path at every collocation point, and a Monte Carlo estimate of the
same expectation; and of the sparse-grid interpolant in the local variables:
nodal reproduction, the Smolyak polynomial space, the one-variable Lagrange
interpolant, convergence beyond the tensor grid, and the plain path outside
the box."""
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


# ---- sparse-grid interpolation in the local variables ----
@pytest.mark.parametrize("k,level", [(1, 3), (2, 3), (3, 2), (4, 2)])
def test_interpolant_reproduces_nodal_values(k, level):
    # nested nodes: the Smolyak interpolant is an interpolant
    dg, _ = sc.sparse_grid(k, level)
    rng = np.random.default_rng(k * 10 + level)
    vals = {tuple(int(v) for v in r): rng.normal(size=3) for r in dg}
    t = np.cos(np.pi * dg / sc.digit_base(level))
    got = sc.smolyak_interp(vals, k, level, t)
    np.testing.assert_allclose(got, [vals[tuple(int(v) for v in r)] for r in dg], rtol=0, atol=1e-13)


def _min_level(a):
    # lowest nested level whose node count exceeds the degree a
    i = 1
    while sc.cc_npoints(i) - 1 < a:
        i += 1
    return i


@pytest.mark.parametrize("k,level", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_interpolant_polynomial_exactness(k, level):
    # exact on x^a whenever sum_d (level(a_d) - 1) <= L, the Smolyak space
    # (Barthelmann, Novak and Ritter); not exact just outside it
    import itertools
    dg, _ = sc.sparse_grid(k, level)
    X = np.cos(np.pi * dg / sc.digit_base(level))
    t = np.random.default_rng(3).uniform(-1, 1, size=(40, k))
    for a in itertools.product(range(10), repeat=k):
        need = sum(_min_level(ad) - 1 for ad in a)
        if need > level + 1:
            continue
        vals = {tuple(int(v) for v in r): np.array([np.prod(x ** np.array(a))]) for r, x in zip(dg, X)}
        err = np.abs(sc.smolyak_interp(vals, k, level, t)[:, 0] - np.prod(t ** np.array(a), axis=1)).max()
        if need <= level:
            assert err < 1e-12, (a, err)
        elif sum(a) == max(a):  # one variable of too high a degree
            assert err > 1e-6, (a, err)


def test_one_variable_is_the_lagrange_interpolant_on_the_finest_nodes():
    dg, _ = sc.sparse_grid(1, 3)
    x = np.cos(np.pi * dg[:, 0] / 8)
    f = np.exp(x) * np.sin(3 * x)
    vals = {(int(d),): np.array([v]) for d, v in zip(dg[:, 0], f)}
    t = np.linspace(-1, 1, 37)
    ref = np.polyval(np.polyfit(x, f, len(x) - 1), t)
    np.testing.assert_allclose(sc.smolyak_interp(vals, 1, 3, t[:, None])[:, 0], ref, rtol=0, atol=1e-12)


def test_interpolant_of_the_patch_stiffness_converges_faster_than_the_tensor_grid():
    # a patch with four local variables of the 8x8 mesh: level 4 (401 nodes)
    # beats the 5^4 = 625-node tensor interpolant, and levels 2..5 converge
    from oracle import ri
    wl = W.MESH8
    fam = _fam()
    lv = ri.local_vars_bumps(wl.nc, wl.m, fam["g"], fam["rho"])
    K = [i for i, l in enumerate(lv) if len(l) == 4][0]
    only = [lv[K] if k == K else [] for k in range(wl.M)]
    xi = np.zeros((100, wl.nxi))
    xi[:, lv[K]] = np.random.default_rng(5).uniform(-1, 1, size=(100, 4))
    Sref = ri.patch_S(xi, K, wl.nc, wl.m, fam)
    err = {}
    for L in (2, 3, 4, 5):
        model = sc.sgi_offline(wl.nc, wl.m, fam, only, L)
        S = sc.smolyak_interp(model["tables"][K], 4, L, xi[:, lv[K]])
        err[L] = np.abs(S - Sref).max() / np.abs(Sref).max()
    assert err[2] > err[3] > err[4] > err[5] and err[5] < 1e-9, err
    tens = ri.ri_offline(wl.nc, wl.m, fam, lv, 5, -1, 1, patches=[K])
    et = np.abs(ri.ri_eval(tens["tables"][K], tens["nodes"], xi[:, lv[K]]) - Sref).max() / np.abs(Sref).max()
    assert err[4] < 0.1 * et, (err[4], et)


def test_interpolation_outside_the_box_is_the_plain_path():
    from oracle import core, ri
    wl = W.MESH8
    fam = _fam()
    lv = ri.local_vars_bumps(wl.nc, wl.m, fam["g"], fam["rho"])
    model = sc.sgi_offline(wl.nc, wl.m, fam, lv, 2, lo=-0.5, hi=0.5)
    xi = W.uniform_xi(6, wl.nxi, 31)
    S, fb = sc.sgi_online(model, xi, wl.nc, wl.m, fam)
    a = core.coef_bumps(xi, wl.nfine, **fam)
    Sp, _, _ = core.upscale(a, wl.nc, wl.nc, wl.m)
    assert fb.any() and (~fb).any()
    np.testing.assert_array_equal(S[fb], Sp[fb])
    assert np.abs(S[~fb] - Sp[~fb]).max() < 0.05 * np.abs(Sp).max()
