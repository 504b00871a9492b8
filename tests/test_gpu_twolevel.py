"""Fine-grid FEM and the two-level Monte Carlo estimator on the GPU (Sec.
4.1.1, the remark with eqs. MCmean2level and mseML) against the oracle:
fine solutions on meshes of 2..64 cells per side (several chunks of samples
at 64), the status of a failed solve, the estimator's mean and variances,
and the estimator at the throughput shape of the 8x8 mesh; the
multigrid-preconditioned CG fine solver on meshes up to 256 cells per side
(odd coarsest levels included) against the oracle's direct solve, and the
two-level estimator on a 128 x 128 fine mesh; the control-variate estimator
of the remark closing Sec. 5.3 (the same formula with the plain coarse
solution in place of the fine one) against the oracle.

PCG tolerances: relative residual 1e-13 (bump coefficients) or 1e-14 (four
decades); the solution error is at most the condition number times that, in
practice far below: 1e-9 and 1e-8 relative per sample are asserted.

Tolerances: fine solutions 1e-10 relative per sample (FP64 banded
factorisations on both sides, different elimination order); the estimator
sums FP64 values in a different order: mean 1e-10 relative, variances
(differences of two sums) 1e-8 relative plus 1e-14 max|u|^2."""
import sys

import numpy as np
import pytest
import torch

from oracle import core, twolevel
from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


def say(msg):
    print(f"[gpu-2l] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem
    assert torch.cuda.is_available()
    stomsfem.lib()
    return stomsfem


def _rel(u, ref):
    return (np.linalg.norm(u - ref, axis=-1) / np.linalg.norm(ref, axis=-1)).max()


@pytest.mark.parametrize("nf,N", [(2, 3), (8, 5), (24, 3), (64, 2)])
def test_fine_solve_matches_oracle(sm, nf, N):
    say(f"fine solve nf={nf} N={N}")
    a = W.uniform_array((N, nf, nf), 0.2, 5.0, 1800 + nf)
    a[-1] = np.exp(W.uniform_array((nf, nf), -4.6, 4.6, 1900 + nf))  # four decades
    u = sm.fine_solve(torch.from_numpy(a).cuda()).cpu().numpy()
    ref = twolevel.fine_solutions(a)
    err = _rel(u, ref)
    say(f"  rel err {err:.2e}")
    assert err <= TOL


def test_fine_solve_over_several_chunks(sm):
    # 420 samples at 64 x 64 exceed one chunk of samples (409)
    nf, N = 64, 420
    say(f"fine solve nf={nf} N={N}")
    wl = W.MESH8
    xi = W.uniform_xi(N, wl.nxi, 1810)
    a = sm.coef_bumps(torch.from_numpy(xi).cuda(), wl.nfine, **wl.coef_params())
    st = torch.full((N,), 99, dtype=torch.int32, device="cuda")
    u = sm.fine_solve(a, status=st).cpu().numpy()
    assert int(st.abs().sum()) == 0
    pick = [0, 1, 408, 409, 410, N - 1]
    a_ref = core.coef_bumps(xi[pick], wl.nfine, **wl.coef_params())
    assert _rel(u[pick], twolevel.fine_solutions(a_ref)) <= TOL


def test_fine_solve_flags_a_failed_sample(sm):
    a = W.uniform_array((3, 16, 16), 0.5, 2.0, 1820)
    a[1] = -a[1]
    st = torch.full((3,), 99, dtype=torch.int32, device="cuda")
    sm.fine_solve(torch.from_numpy(a).cuda(), status=st)
    st = st.cpu().numpy()
    assert st[0] == 0 and st[2] == 0 and st[1] == sm.ENOTSPD


def _coarse(sm, wl, xi):
    a = sm.coef_bumps(xi, wl.nfine, **wl.coef_params())
    U, _, _ = sm.coarse_solve(sm.upscale(a, wl.nc, wl.nc, wl.m), wl.nc, wl.nc)
    return a, U


def _oracle_coarse(wl, xi):
    a = core.coef_bumps(xi, wl.nfine, **wl.coef_params())
    S, _, _ = core.upscale(a, wl.nc, wl.nc, wl.m)
    U, _, _ = core.coarse_solve(S, wl.nc, wl.nc)
    return a, U


@pytest.mark.parametrize("nH,nh", [(300, 40), (16384, 512)])
def test_two_level_matches_oracle(sm, nH, nh):
    # 16384 / 512: the throughput shape of the 8x8 mesh, in the launch
    # configuration of the benchmark
    wl = W.MESH8
    say(f"two-level nH={nH} nh={nh}")
    xH = W.uniform_xi(nH, wl.nxi, 1830)
    xh = W.uniform_xi(nh, wl.nxi, 1831)
    _, U_H = _coarse(sm, wl, torch.from_numpy(xH).cuda())
    a_h, U_Hh = _coarse(sm, wl, torch.from_numpy(xh).cuda())
    u_f = sm.fine_solve(a_h)
    mean, var_H, var_d = [t.cpu().numpy() for t in sm.two_level_mc(U_H, U_Hh, u_f, wl.nc, wl.m)]
    _, U_H_ref = _oracle_coarse(wl, xH)
    a_h_ref, U_Hh_ref = _oracle_coarse(wl, xh)
    m_ref, vH_ref, vd_ref, _ = twolevel.two_level(U_H_ref, U_Hh_ref, twolevel.fine_solutions(a_h_ref), wl.nc, wl.m)
    umax = np.abs(U_H_ref).max()
    np.testing.assert_allclose(mean, m_ref, rtol=1e-10, atol=0)
    np.testing.assert_allclose(var_H, vH_ref, rtol=1e-8, atol=1e-14 * umax**2)
    np.testing.assert_allclose(var_d, vd_ref, rtol=1e-8, atol=1e-14 * umax**2)


def test_invalid_arguments(sm):
    with pytest.raises(sm.StomsfemError):  # beyond the largest fine mesh (no samples, nothing allocated)
        sm.fine_solve(torch.zeros((0, 8193, 8193), dtype=torch.float64, device="cuda"))
    with pytest.raises(sm.StomsfemError):
        sm.fine_solve_pcg(torch.zeros((1, 8, 8), dtype=torch.float64, device="cuda"), tol=0.0)
    with pytest.raises(sm.StomsfemError):
        sm.fine_solve(torch.zeros((1, 1, 1), dtype=torch.float64, device="cuda"))
    z = torch.zeros((0, 49), dtype=torch.float64, device="cuda")
    with pytest.raises(sm.StomsfemError):  # empty sample sets
        sm.two_level_mc(z, z, torch.zeros((0, 63 * 63), dtype=torch.float64, device="cuda"), 8, 8)
    assert sm.fine_solve(torch.zeros((0, 8, 8), dtype=torch.float64, device="cuda")).shape == (0, 49)


@pytest.mark.parametrize("nf,N", [(16, 3), (96, 2), (128, 3), (256, 1)])
def test_fine_solve_pcg_matches_oracle(sm, nf, N):
    # bump-family samples on an nf x nf fine mesh (the 32x32 workload's
    # geometry) plus, for N > 1, a last sample with four decades of element-wise
    # independent contrast; 96 = 3 * 32 ends on an odd coarsest level
    wl = W.MESH32
    say(f"fine PCG nf={nf} N={N}")
    xi = W.uniform_xi(N, wl.nxi, 1840 + nf)
    a = core.coef_bumps(xi, nf, **wl.coef_params())
    if N > 1:
        a[-1] = np.exp(W.uniform_array((nf, nf), -4.6, 4.6, 1940 + nf))
    u, it, st = sm.fine_solve_pcg(torch.from_numpy(a).cuda(), tol=1e-14 if N > 1 else 1e-13)
    torch.cuda.synchronize()
    ref = twolevel.fine_solutions(a)
    u = u.cpu().numpy()
    err_b = _rel(u[: max(1, N - 1)], ref[: max(1, N - 1)])
    say(f"  iterations {it.cpu().numpy().tolist()}, status {st.cpu().numpy().tolist()}, bump rel err {err_b:.2e}")
    assert (st.cpu().numpy() == 0).all()
    assert err_b <= 1e-9
    if N > 1:
        err_c = _rel(u[-1:], ref[-1:])
        say(f"  four-decade rel err {err_c:.2e}")
        assert err_c <= 1e-8


def test_fine_solve_dispatches_to_pcg_beyond_64(sm):
    # stomsfem_fine_solve takes the PCG path above 64 cells per side
    wl = W.MESH32
    nf = 128
    xi = W.uniform_xi(2, wl.nxi, 1851)
    a = torch.from_numpy(core.coef_bumps(xi, nf, **wl.coef_params())).cuda()
    st = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    u = sm.fine_solve(a, status=st)
    u2, _, _ = sm.fine_solve_pcg(a)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    assert torch.equal(u, u2)


def test_two_level_on_a_128_fine_mesh_matches_oracle(sm):
    # 8 x 8 coarse elements of 16 x 16 fine cells (fine mesh 128 x 128, the
    # 32x32 workload's bump geometry), fine solutions by PCG
    wl = W.MESH32
    nc, m = 8, 16
    nH, nh = 64, 6
    say(f"two-level on a {nc * m} fine mesh: nH={nH} nh={nh}")
    xH = W.uniform_xi(nH, wl.nxi, 1860)
    xh = W.uniform_xi(nh, wl.nxi, 1861)
    cp = wl.coef_params()
    aH = core.coef_bumps(xH, nc * m, **cp)
    ah = core.coef_bumps(xh, nc * m, **cp)
    S_H = sm.upscale(torch.from_numpy(aH).cuda(), nc, nc, m)
    S_h = sm.upscale(torch.from_numpy(ah).cuda(), nc, nc, m)
    U_H, _, _ = sm.coarse_solve(S_H, nc, nc)
    U_Hh, _, _ = sm.coarse_solve(S_h, nc, nc)
    u_f, _, st = sm.fine_solve_pcg(torch.from_numpy(ah).cuda(), tol=1e-13)
    mean, var_H, var_d = [t.cpu().numpy() for t in sm.two_level_mc(U_H, U_Hh, u_f, nc, m)]
    assert (st.cpu().numpy() == 0).all()
    SH_ref, _, _ = core.upscale(aH, nc, nc, m)
    Sh_ref, _, _ = core.upscale(ah, nc, nc, m)
    UH_ref, _, _ = core.coarse_solve(SH_ref, nc, nc)
    UHh_ref, _, _ = core.coarse_solve(Sh_ref, nc, nc)
    m_ref, vH_ref, vd_ref, _ = twolevel.two_level(UH_ref, UHh_ref, twolevel.fine_solutions(ah), nc, m)
    umax = np.abs(UH_ref).max()
    np.testing.assert_allclose(mean, m_ref, rtol=1e-9, atol=0)
    np.testing.assert_allclose(var_H, vH_ref, rtol=1e-8, atol=1e-14 * umax**2)
    np.testing.assert_allclose(var_d, vd_ref, rtol=1e-6, atol=1e-13 * umax**2)


def test_control_variate_estimator_matches_oracle(sm):
    # the remark closing Sec. 5.3: the accelerated coarse solution u^_H on a
    # large sample set corrected by M[u_H - u^_H] on a small one; here u^_H is
    # the reduced-basis solution of the 8x8 mesh and u_H the plain one.  It is
    # the two-level formula with the plain coarse nodal values in place of the
    # fine ones (m = 1: the fine node of a coarse node is the node itself).
    wl = W.MESH8
    n1, n2 = 2000, 100
    xi_tr = torch.from_numpy(W.uniform_xi(64, wl.nxi, 2863)).cuda()
    model = sm.reduce(sm.coef_bumps(xi_tr, wl.nfine, **wl.coef_params()), wl.nc, wl.nc, wl.m)
    x1 = W.uniform_xi(n1, wl.nxi, 1862)
    x2 = W.uniform_xi(n2, wl.nxi, 1863)
    a1 = sm.coef_bumps(torch.from_numpy(x1).cuda(), wl.nfine, **wl.coef_params())
    a2 = sm.coef_bumps(torch.from_numpy(x2).cuda(), wl.nfine, **wl.coef_params())
    U1_acc, _, _ = sm.coarse_solve(sm.reduce_apply(model, a1, precision=sm.PREC_F32), wl.nc, wl.nc)
    U2_acc, _, _ = sm.coarse_solve(sm.reduce_apply(model, a2, precision=sm.PREC_F32), wl.nc, wl.nc)
    U2_pl, _, _ = sm.coarse_solve(sm.upscale(a2, wl.nc, wl.nc, wl.m), wl.nc, wl.nc)
    mean, var_1, var_d = [t.cpu().numpy() for t in sm.two_level_mc(U1_acc, U2_acc, U2_pl, wl.nc, 1)]
    m_ref, v1_ref, vd_ref, _ = twolevel.two_level(U1_acc.cpu().numpy(), U2_acc.cpu().numpy(), U2_pl.cpu().numpy(),
                                                  wl.nc, 1)
    umax = float(U1_acc.abs().max())
    np.testing.assert_allclose(mean, m_ref, rtol=1e-12, atol=0)
    np.testing.assert_allclose(var_1, v1_ref, rtol=1e-9, atol=1e-15 * umax**2)
    np.testing.assert_allclose(var_d, vd_ref, rtol=1e-6, atol=1e-15 * umax**2)
    say(f"control variate: var[u_H - u^_H] / var[u^_H] = {float(var_d.sum() / var_1.sum()):.2e}")
    assert var_d.sum() < 1e-3 * var_1.sum()
    model.free()
