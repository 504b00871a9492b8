"""Fine-grid FEM and the two-level Monte Carlo estimator on the GPU (Sec.
4.1.1, the remark with eqs. MCmean2level and mseML) against the oracle:
fine solutions on meshes of 2..64 cells per side (several chunks of samples
at 64), the status of a failed solve, the estimator's mean and variances,
and the estimator at the throughput shape of the 8x8 mesh.

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
    with pytest.raises(sm.StomsfemError):
        sm.fine_solve(torch.zeros((1, 65, 65), dtype=torch.float64, device="cuda"))
    with pytest.raises(sm.StomsfemError):
        sm.fine_solve(torch.zeros((1, 1, 1), dtype=torch.float64, device="cuda"))
    z = torch.zeros((0, 49), dtype=torch.float64, device="cuda")
    with pytest.raises(sm.StomsfemError):  # empty sample sets
        sm.two_level_mc(z, z, torch.zeros((0, 63 * 63), dtype=torch.float64, device="cuda"), 8, 8)
    assert sm.fine_solve(torch.zeros((0, 8, 8), dtype=torch.float64, device="cuda")).shape == (0, 49)
