"""Sparse-grid stochastic collocation with search-and-plug-in dictionaries on
the GPU (Sec. 4.1.2, global SC methods; Sec. 5.2) against
the oracle: the dictionaries' S at every collocation point, the weighted
quadrature, the end-to-end mean and variance, points missing from a
dictionary, and sampled points of the level-4 grid in 16 variables.

Tolerances: S and U 1e-10 relative (FP64 cell and coarse solves on both
sides, the plain-path bound); the quadrature's weighted sums of U are formed
in different orders with weights of both signs up to ~2 in size, so the
mean agrees to 1e-10 relative and the variance (a difference of two sums)
to 1e-7 relative plus 1e-12 max|mean|^2."""
import sys

import numpy as np
import pytest
import torch

from oracle import core, ri, sc
from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


def say(msg):
    print(f"[gpu-sc] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem
    assert torch.cuda.is_available()
    stomsfem.lib()
    return stomsfem


SC16 = W.BumpWorkload("sc_mesh4_h16", nc=4, m=16, nsamples=1, g=3, rho=0.25, eps=1.0 / 32, seed=1501)


def _setup(sm, wl):
    fam = sm.bump_family(wl)
    lv, nl = sm.local_vars_bumps(wl.nc, wl.nc, wl.m, fam)
    lv_orc = ri.local_vars_bumps(wl.nc, wl.m, wl.g, wl.rho)
    assert [list(r[:n]) for r, n in zip(lv, nl)] == lv_orc
    return fam, lv, lv_orc


def _relerr(S, Sref):
    return (np.abs(S - Sref).max(-1) / np.abs(Sref).max(-1)).max()


@pytest.mark.parametrize("wl,level", [(W.MESH8, 1), (W.MESH8, 2), (SC16, 3)])
def test_plug_in_matches_the_plain_path(sm, wl, level):
    say(f"{wl.name} level {level}")
    fam, lv, lv_orc = _setup(sm, wl)
    dg, w = sm.sparse_grid(wl.nxi, level)
    model = sm.sc_build(wl.nc, wl.nc, wl.m, lv, fam, level, dg)
    st = torch.full((len(w), wl.M), 99, dtype=torch.int32, device="cuda")
    S = sm.sc_apply(model, torch.from_numpy(dg).cuda(), status=st)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    S_ref = sc.sc_direct(wl.nc, wl.m, wl.coef_params(), dg.astype(np.int64), level)
    err = _relerr(S.cpu().numpy(), S_ref)
    say(f"  {len(w)} points, S rel err {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("level", [2, 3])
def test_end_to_end_mean_and_variance(sm, level):
    wl = W.MESH8
    say(f"end to end level {level}")
    fam, lv, lv_orc = _setup(sm, wl)
    dg, w = sm.sparse_grid(wl.nxi, level)
    model = sm.sc_build(wl.nc, wl.nc, wl.m, lv, fam, level, dg)
    S = sm.sc_apply(model, torch.from_numpy(dg).cuda())
    U, _, _ = sm.coarse_solve(S, wl.nc, wl.nc)
    mean, var = sm.quadrature(U, torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    orc_model = sc.sc_offline(wl.nc, wl.m, wl.coef_params(), lv_orc, dg.astype(np.int64), level)
    dr, wr = sc.sparse_grid(wl.nxi, level)
    U_ref, _, _ = core.coarse_solve(sc.sc_plug_in(orc_model, dr), wl.nc, wl.nc)
    mean_ref, var_ref = sc.quadrature(U_ref, wr)
    U = U.cpu().numpy()
    err = (np.linalg.norm(U - U_ref, axis=1) / np.linalg.norm(U_ref, axis=1)).max()
    say(f"  U rel err {err:.2e}")
    assert err <= TOL
    np.testing.assert_allclose(mean.cpu().numpy(), mean_ref, rtol=1e-10, atol=0)
    np.testing.assert_allclose(var.cpu().numpy(), var_ref, rtol=1e-7, atol=1e-12 * np.abs(mean_ref).max() ** 2)


def test_points_missing_from_the_dictionary(sm):
    # dictionaries of the level-1 grid hold local points with at most one
    # variable off the midpoint; a point with two such variables local to a
    # patch is not found there (status 1, NaN) and is found everywhere else
    wl = W.MESH8
    fam, lv, lv_orc = _setup(sm, wl)
    dg, _ = sm.sparse_grid(wl.nxi, 1)
    model = sm.sc_build(wl.nc, wl.nc, wl.m, lv, fam, 1, dg)
    q = np.full((2, wl.nxi), 1, dtype=np.int32)
    q[1, 0] = 0
    q[1, 1] = 2  # variables 0 and 1 off the midpoint
    st = torch.full((2, wl.M), 99, dtype=torch.int32, device="cuda")
    S = sm.sc_apply(model, torch.from_numpy(q).cuda(), status=st).cpu().numpy()
    st = st.cpu().numpy()
    assert (st[0] == 0).all()
    both = np.array([0 in l and 1 in l for l in lv_orc])
    assert both.any() and (~both).any()
    assert (st[1][both] == 1).all() and (st[1][~both] == 0).all()
    assert np.isnan(S[1][both]).all() and np.isfinite(S[1][~both]).all()
    # digits outside 0..D are never found
    q[0, 5] = 7
    st = torch.full((1, wl.M), 99, dtype=torch.int32, device="cuda")
    sm.sc_apply(model, torch.from_numpy(q[:1].copy()).cuda(), status=st)
    st = st.cpu().numpy()[0]
    assert (st[[5 in l for l in lv_orc]] == 1).all() and (st[[5 not in l for l in lv_orc]] == 0).all()


@pytest.mark.parametrize("n,nu", [(1, 1), (257, 49), (1000, 130), (300001, 7)])
def test_quadrature_against_plain_sums(sm, n, nu):
    rng = np.random.default_rng(n + nu)
    U = rng.normal(size=(n, nu)) + 3.0
    w = rng.normal(size=n)
    mean, var = sm.quadrature(torch.from_numpy(U).cuda(), torch.from_numpy(w).cuda())
    mean_ref = np.einsum("p,pi->i", w, U)
    var_ref = np.einsum("p,pi->i", w, U * U) - mean_ref**2
    scale = np.abs(w) @ (U * U)
    assert np.all(np.abs(mean.cpu().numpy() - mean_ref) <= 1e-13 * (np.abs(w) @ np.abs(U)))
    assert np.all(np.abs(var.cpu().numpy() - var_ref) <= 1e-13 * scale + 1e-13 * mean_ref**2)
    # bitwise reproducible
    mean2, var2 = sm.quadrature(torch.from_numpy(U).cuda(), torch.from_numpy(w).cuda())
    assert torch.equal(mean, mean2) and torch.equal(var, var2)


def test_full_size_sampled(sm):
    # the collocation workload of the benchmark (8 x 8 mesh, H/h = 8, 16
    # variables, level 4: 51 137 points): grid against the oracle's, and the
    # plugged-in S and coarse solutions of sampled points against the plain
    # path at those points
    wl = W.MESH8
    level = 4
    say(f"full size level {level}")
    fam, lv, lv_orc = _setup(sm, wl)
    dg, w = sm.sparse_grid(wl.nxi, level)
    dr, wr = sc.sparse_grid(wl.nxi, level)
    assert (dg == dr).all()
    np.testing.assert_allclose(w, wr, rtol=0, atol=1e-10)
    model = sm.sc_build(wl.nc, wl.nc, wl.m, lv, fam, level, dg)
    st = torch.full((len(w), wl.M), 99, dtype=torch.int32, device="cuda")
    S = sm.sc_apply(model, torch.from_numpy(dg).cuda(), status=st)
    U, _, _ = sm.coarse_solve(S, wl.nc, wl.nc)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    pick = np.random.default_rng(11).choice(len(w), 200, replace=False)
    S_ref = sc.sc_direct(wl.nc, wl.m, wl.coef_params(), dr[pick], level)
    assert _relerr(S.cpu().numpy()[pick], S_ref) <= TOL
    U_ref, _, _ = core.coarse_solve(S_ref, wl.nc, wl.nc)
    Ug = U.cpu().numpy()[pick]
    assert (np.linalg.norm(Ug - U_ref, axis=1) / np.linalg.norm(U_ref, axis=1)).max() <= TOL


def test_invalid_arguments(sm):
    wl = W.MESH8
    fam, lv, _ = _setup(sm, wl)
    dg, _ = sm.sparse_grid(wl.nxi, 1)
    model = sm.sc_build(wl.nc, wl.nc, wl.m, lv, fam, 1, dg)
    with pytest.raises(sm.StomsfemError):  # host digits
        sm.lib()
        import ctypes as C
        S = torch.empty((len(dg), wl.M, 10), dtype=torch.float64, device="cuda")
        sm._check("stomsfem_sc_apply", sm.lib().stomsfem_sc_apply(
            model.handle, dg.ctypes.data_as(C.c_void_p), wl.nxi, len(dg), sm._ptr(S), None, None))
    with pytest.raises(sm.StomsfemError):  # fewer digit columns than variables
        sm.sc_apply(model, torch.from_numpy(dg[:, :8].copy()).cuda())
    with pytest.raises(sm.StomsfemError):  # not a collocation model
        rb = sm.interp_build(wl.nc, wl.nc, wl.m, lv, fam, 2)
        sm.sc_apply(rb, torch.from_numpy(dg).cuda())
    with pytest.raises(sm.StomsfemError):
        model.save("/tmp/stomsfem_sc_model.bin")
    assert sm.sc_apply(model, torch.zeros((0, wl.nxi), dtype=torch.int32, device="cuda")).shape == (0, wl.M, 10)
