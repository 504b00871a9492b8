"""GPU parity of the plain FP64 path (through the C-ABI) against the CPU oracle.

Tolerances (FP64 path): per (element, sample) pair,
max_q |S_q - S_q^ref| <= 1e-10 * max_q |S_q^ref|; per sample,
||U - U^ref||_2 <= 1e-10 ||U^ref||_2.  Both sides solve SPD systems whose
condition numbers are below 1e5 here, so a correct FP64 implementation lands
near 1e-13; 1e-10 leaves room for the different elimination orders.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu

STOL = 1e-10
UTOL = 1e-10


def say(msg):
    print(f"[gpu-plain] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem

    assert torch.cuda.is_available()
    stomsfem.lib()
    return stomsfem


def s_relerr(S, Sref):
    S, Sref = np.asarray(S), np.asarray(Sref)
    return (np.abs(S - Sref).max(-1) / np.abs(Sref).max(-1)).max()


def u_relerr(U, Uref):
    return (np.linalg.norm(U - Uref, axis=-1) / np.linalg.norm(Uref, axis=-1)).max()


@pytest.mark.parametrize("nfine,g,rho", [(100, 3, 0.3), (40, 3, 0.2), (24, 2, 0.4), (64, 4, 0.25), (256, 8, 0.125),
                                         (1024, 8, 0.125), (96, 3, 0.1)])
def test_coefficients_on_tiles_inside_and_across_bump_cells(sm, orc, nfine, g, rho):
    # bump cells of 33.3, 13.3, 12, 16, 32, 128 (the benchmark mesh) and 32
    # elements: 16 x 16 tiles that lie in one cell (where the bumps whose disc
    # misses the tile are skipped; rho = 0.1 leaves some tiles with only their
    # own cell's bump) and tiles that straddle two, partial tiles at the edge,
    # FP64 and FP32 storage
    xi = W.uniform_xi(3, g * g, 1950 + nfine)
    prm = dict(g=g, rho=rho, eps=1.0 / 32, base=2.0, amp=1.8, beta=0.5)
    a_ref = orc.coef_bumps(xi, nfine, **prm)
    a = sm.coef_bumps(torch.from_numpy(xi).cuda(), nfine, **prm)
    a32 = sm.coef_bumps(torch.from_numpy(xi).cuda(), nfine, dtype=torch.float32, **prm)
    torch.cuda.synchronize()
    np.testing.assert_allclose(a.cpu().numpy(), a_ref, rtol=1e-14, atol=0)
    np.testing.assert_allclose(a32.cpu().numpy(), a_ref.astype(np.float32), rtol=1e-7, atol=0)


def test_mesh8_end_to_end(sm, orc):
    wl = W.MESH8
    say(f"mesh8 end to end: N={wl.nsamples} nc={wl.nc} m={wl.m}")
    xi = W.uniform_xi(wl.nsamples, wl.nxi, wl.seed)
    a_ref = orc.coef_bumps(xi, wl.nfine, **wl.coef_params())
    xi_d = torch.from_numpy(xi).cuda()
    a = sm.coef_bumps(xi_d, wl.nfine, **wl.coef_params())
    torch.cuda.synchronize()
    np.testing.assert_allclose(a.cpu().numpy(), a_ref, rtol=1e-14, atol=0)
    status = torch.full((wl.nsamples, wl.M), 99, dtype=torch.int32, device="cuda")
    S = sm.upscale(a, wl.nc, wl.nc, wl.m, status=status)
    U, mean, var = sm.coarse_solve(S, wl.nc, wl.nc)
    torch.cuda.synchronize()
    S_ref, _, _ = orc.upscale(a_ref, wl.nc, wl.nc, wl.m)
    U_ref, mean_ref, var_ref = orc.coarse_solve(S_ref, wl.nc, wl.nc)
    assert (status.cpu().numpy() == 0).all()
    assert s_relerr(S.cpu().numpy(), S_ref) < STOL
    assert u_relerr(U.cpu().numpy(), U_ref) < UTOL
    np.testing.assert_allclose(mean.cpu().numpy(), mean_ref, rtol=UTOL)
    np.testing.assert_allclose(var.cpu().numpy(), var_ref, rtol=1e-8, atol=1e-12 * np.abs(mean_ref).max() ** 2)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7, 8])
def test_small_m_ragged(sm, orc, m):
    # ncx != ncy, a pair count that is not a multiple of the 64-lane wavefront,
    # log-normal coefficients spanning about four decades
    ncx, ncy, N = 3, 5, 7
    say(f"small m ragged: m={m} ncx={ncx} ncy={ncy} N={N}")
    a_np = W.lognormal_field((N, ncy * m, ncx * m), 1.5, 500 + m)
    a = torch.from_numpy(a_np).cuda()
    S = sm.upscale(a, ncx, ncy, m)
    torch.cuda.synchronize()
    S_ref, _, _ = orc.upscale(a_np, ncx, ncy, m)
    assert s_relerr(S.cpu().numpy(), S_ref) < STOL


@pytest.mark.parametrize("m", [8, 12, 16, 32])
def test_reference_kernel(sm, orc, m):
    ncx, ncy, N = 2, 3, 2
    say(f"reference kernel: m={m} ncx={ncx} ncy={ncy} N={N}")
    a_np = W.lognormal_field((N, ncy * m, ncx * m), 1.0, 600 + m)
    a = torch.from_numpy(a_np).cuda()
    S = sm.upscale_reference(a, ncx, ncy, m)
    torch.cuda.synchronize()
    S_ref, _, _ = orc.upscale(a_np, ncx, ncy, m)
    assert s_relerr(S.cpu().numpy(), S_ref) < STOL


@pytest.mark.parametrize("m", [8, 16, 32])
def test_dispatch_kernel_matches_oracle(sm, orc, m):
    ncx, ncy, N = 4, 3, 3
    say(f"dispatch kernel: m={m} ncx={ncx} ncy={ncy} N={N}")
    a_np = W.lognormal_field((N, ncy * m, ncx * m), 1.0, 700 + m)
    a = torch.from_numpy(a_np).cuda()
    S = sm.upscale(a, ncx, ncy, m)
    torch.cuda.synchronize()
    S_ref, _, _ = orc.upscale(a_np, ncx, ncy, m)
    assert s_relerr(S.cpu().numpy(), S_ref) < STOL


def test_float32_coefficients(sm, orc):
    # FP32 coefficient storage: the solve is still FP64 on the widened values
    m, nc, N = 8, 3, 4
    say("float32 coefficients")
    a32 = W.lognormal_field((N, nc * m, nc * m), 1.0, 800).astype(np.float32)
    S = sm.upscale(torch.from_numpy(a32).cuda(), nc, nc, m)
    torch.cuda.synchronize()
    S_ref, _, _ = orc.upscale(a32.astype(np.float64), nc, nc, m)
    assert s_relerr(S.cpu().numpy(), S_ref) < STOL


def test_bad_pivot_flags_only_that_pair(sm):
    m, nc, N = 8, 2, 3
    say("non-positive coefficient status")
    a_np = W.lognormal_field((N, nc * m, nc * m), 0.5, 900)
    a_np[1, 3, 12] = -50.0       # sample 1, element K=(1,0)
    a_np[2, 9, 2] = np.nan       # sample 2, element K=(0,1)
    a = torch.from_numpy(a_np).cuda()
    st = torch.full((N, nc * nc), 99, dtype=torch.int32, device="cuda")
    sm.upscale(a, nc, nc, m, status=st)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    expect = np.zeros_like(st)
    expect[1, 1] = sm.ENOTSPD
    expect[2, 2] = sm.ENOTSPD
    np.testing.assert_array_equal(st, expect)


def test_empty_and_invalid_arguments(sm):
    say("empty and invalid arguments")
    a = torch.empty((0, 16, 16), dtype=torch.float64, device="cuda")
    S = sm.upscale(a, 2, 2, 8)
    assert S.shape == (0, 4, 10)
    with pytest.raises(sm.StomsfemError) as e:
        sm.upscale(torch.ones((1, 16, 16), dtype=torch.float64, device="cuda"), 2, 2, 8, precision=7)
    assert e.value.code == sm.EINVAL
    # host memory is rejected before anything is queued
    a_host = torch.ones((1, 16, 16), dtype=torch.float64)
    S_dev = torch.empty((1, 4, 10), dtype=torch.float64, device="cuda")
    b = sm.Batch(2, 2, 8, sm.F64, 1, a_host.data_ptr(), S_dev.data_ptr(), None)
    import ctypes
    rc = sm.lib().stomsfem_upscale(ctypes.byref(b), 1, sm.PREC_F64, sm.BC_LINEAR, None)
    assert rc == sm.EINVAL


@pytest.mark.parametrize("ncx,ncy", [(2, 2), (5, 3), (3, 7), (16, 16), (33, 33), (40, 36), (64, 64), (50, 3),
                                     (37, 2), (66, 20)])
def test_coarse_solve(sm, orc, ncx, ncy):
    N, m = 5, 4
    say(f"coarse solve ncx={ncx} ncy={ncy}")
    a_np = W.lognormal_field((N, ncy * m, ncx * m), 1.0, 1000 + ncx * 10 + ncy)
    S_ref, _, _ = orc.upscale(a_np, ncx, ncy, m)
    S = torch.from_numpy(S_ref).cuda()
    load_np = W.uniform_array((ncx * ncy, 4), 0.0, 1.0, 77)
    for load in (None, load_np):
        U, mean, var = sm.coarse_solve(S, ncx, ncy, load=None if load is None else torch.from_numpy(load).cuda())
        torch.cuda.synchronize()
        U_ref, mean_ref, var_ref = orc.coarse_solve(S_ref, ncx, ncy, load_vec=load)
        assert u_relerr(U.cpu().numpy(), U_ref) < UTOL
        np.testing.assert_allclose(mean.cpu().numpy(), mean_ref, rtol=UTOL, atol=1e-300)


@pytest.mark.parametrize("ncx,ncy", [(1, 1), (5, 3), (16, 16), (64, 64)])
def test_element_loads_match_oracle(sm, ncx, ncy):
    from oracle import loads
    say(f"element loads {ncx}x{ncy}")
    for f in ((2.0, 0.0, 0.0, 1.0), (0.3, -1.2, 0.7, 2.5), (1.0, 0.0, 0.0, 0.0)):
        ref = loads.element_loads_bilinear(ncx, ncy, f)
        got = sm.element_loads(ncx, ncy, f).cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max(), f


def test_coarse_solve_with_the_paper_source(sm, orc):
    # Sec. 5.3's source b = 2 + x1 x2 enters through the element loads; the
    # oracle's coarse solve takes the oracle's loads, the GPU solve the GPU's
    from oracle import loads
    m, nc, N = 4, 6, 3
    say("coarse solve with b = 2 + x1 x2")
    a_np = W.lognormal_field((N, nc * m, nc * m), 1.0, 1300)
    S_ref, _, _ = orc.upscale(a_np, nc, nc, m)
    U_ref, mean_ref, _ = orc.coarse_solve(S_ref, nc, nc, load_vec=loads.element_loads_bilinear(nc, nc, (2, 0, 0, 1)))
    U, mean, _ = sm.coarse_solve(torch.from_numpy(S_ref).cuda(), nc, nc, load=sm.element_loads(nc, nc))
    torch.cuda.synchronize()
    assert u_relerr(U.cpu().numpy(), U_ref) < UTOL
    assert np.abs(mean.cpu().numpy() - mean_ref).max() <= 1e-10 * np.abs(mean_ref).max()
    # the constant source's loads reproduce the default (NULL) load exactly
    U1, _, _ = sm.coarse_solve(torch.from_numpy(S_ref).cuda(), nc, nc, load=sm.element_loads(nc, nc, (1, 0, 0, 0)))
    U0, _, _ = sm.coarse_solve(torch.from_numpy(S_ref).cuda(), nc, nc)
    torch.cuda.synchronize()
    assert u_relerr(U1.cpu().numpy(), U0.cpu().numpy()) < 1e-14
    # argument errors are caught on the host
    import ctypes
    out = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    bad = (ctypes.c_double * 4)(1.0, float("nan"), 0.0, 0.0)
    assert sm.lib().stomsfem_element_loads(2, 2, bad, ctypes.c_void_p(out.data_ptr()), None) == sm.EINVAL
    good = (ctypes.c_double * 4)(1.0, 0.0, 0.0, 0.0)
    assert sm.lib().stomsfem_element_loads(0, 2, good, ctypes.c_void_p(out.data_ptr()), None) == sm.EINVAL
    host = torch.empty((4, 4), dtype=torch.float64)
    assert sm.lib().stomsfem_element_loads(2, 2, good, ctypes.c_void_p(host.data_ptr()), None) == sm.EINVAL
    assert sm.lib().stomsfem_element_loads(2, 2, None, ctypes.c_void_p(out.data_ptr()), None) == sm.EINVAL


def test_coarse_two_by_two_closed_form(sm):
    # nc = 2, S = K_ref (a == 1), f = 1: U = 3/32
    say("coarse 2x2 closed form")
    K = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    Sp = np.array([K[i, j] for (i, j) in [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]])
    S = torch.from_numpy(np.tile(Sp, (3, 4, 1))).cuda()
    U, mean, var = sm.coarse_solve(S, 2, 2)
    torch.cuda.synchronize()
    assert np.abs(U.cpu().numpy() - 3.0 / 32.0).max() < 1e-15
    assert abs(var.cpu().numpy()[0]) < 1e-16


def test_mesh32_full_batch_sampled(sm, orc):
    # the benchmark's configuration: 32 x 32 coarse, H/h = 32, all 4096
    # samples in one batch (34 GB of FP64 coefficients), the autotuned launch;
    # sampled pairs and whole samples against the oracle
    wl = W.MESH32
    xi_np = W.uniform_xi(wl.nsamples, wl.nxi, wl.seed)
    xi = torch.from_numpy(xi_np).cuda()
    a = sm.coef_bumps(xi, wl.nfine, **wl.coef_params())
    S = torch.empty((wl.nsamples, wl.M, 10), dtype=torch.float64, device="cuda")
    rep = sm.autotune(a, wl.nc, wl.nc, wl.m, S=S, reps=1)
    st = torch.full((wl.nsamples, wl.M), -9, dtype=torch.int32, device="cuda")
    sm.upscale(a, wl.nc, wl.nc, wl.m, S=S, status=st)
    U, qm, qv = sm.coarse_solve(S, wl.nc, wl.nc)
    torch.cuda.synchronize()
    say(f"mesh32 full batch: tuned {rep}")
    assert int((st != 0).sum()) == 0
    assert bool(torch.isfinite(S).all()) and bool(torch.isfinite(U).all())
    rng = np.random.default_rng(77)
    samples = [0, wl.nsamples - 1] + rng.choice(wl.nsamples, 2, replace=False).tolist()
    for s in samples:
        a_s = orc.coef_bumps(xi_np[s:s + 1], wl.nfine, **wl.coef_params())
        np.testing.assert_allclose(a[s].cpu().numpy(), a_s[0], rtol=1e-14, atol=0)
        Sr, _, _ = orc.upscale(a_s, wl.nc, wl.nc, wl.m)
        assert s_relerr(S[s].cpu().numpy(), Sr[0]) <= STOL
        Ur, _, _ = orc.coarse_solve(Sr, wl.nc, wl.nc)
        assert u_relerr(U[s:s + 1].cpu().numpy(), Ur) <= UTOL
    # QoI: the sample mean of U over the batch
    np.testing.assert_allclose(qm.cpu().numpy(), U.mean(dim=0).cpu().numpy(), rtol=1e-12, atol=0)
    sm.tuning_reset()
    del a


@pytest.mark.parametrize("m,ncx,ncy", [(2, 3, 2), (5, 2, 3), (8, 4, 4), (13, 2, 2), (16, 3, 2), (32, 2, 2)])
def test_oscillatory_boundary_data_match_oracle(sm, orc, m, ncx, ncy):
    # the oscillatory cell-problem data through the reference kernel (and
    # through stomsfem_upscale, which routes them there) against the oracle's
    # own construction, FP64 and FP32 coefficients
    N = 3
    say(f"oscillatory boundary data m={m} mesh {ncx}x{ncy}")
    a_np = W.lognormal_field((N, ncy * m, ncx * m), 1.5, 3000 + m)
    S_ref, st_ref, _ = orc.upscale(a_np, ncx, ncy, m, bc=orc.BC_OSC)
    assert (st_ref == 0).all()
    a = torch.from_numpy(a_np).cuda()
    S1 = sm.upscale_reference(a, ncx, ncy, m, bc=sm.BC_OSCILLATORY)
    S2 = sm.upscale(a, ncx, ncy, m, bc=sm.BC_OSCILLATORY)
    S_lin = sm.upscale(a, ncx, ncy, m)
    torch.cuda.synchronize()
    for S in (S1, S2):
        Sg = S.cpu().numpy()
        err = np.abs(Sg - S_ref).max(-1) / np.abs(S_ref).max(-1)
        assert err.max() < 1e-10, err.max()
    # the data differ from the linear ones on a heterogeneous medium
    assert (S1 - S_lin).abs().max().item() > 1e-3 * S_lin.abs().max().item()
    a32 = torch.from_numpy(a_np.astype(np.float32)).cuda()
    S32 = sm.upscale(a32, ncx, ncy, m, bc=sm.BC_OSCILLATORY).cpu().numpy()
    S_ref32, _, _ = orc.upscale(a_np.astype(np.float32).astype(np.float64), ncx, ncy, m, bc=orc.BC_OSC)
    assert (np.abs(S32 - S_ref32).max(-1) / np.abs(S_ref32).max(-1)).max() < 1e-10


def test_oscillatory_boundary_data_constant_and_layered(sm, orc):
    # constant coefficient: the oscillatory data are the linear data; media
    # layered across x: the oscillatory S equals the oracle's (whose
    # upscaled x-conductivity is the harmonic mean, pinned on the CPU)
    m, nc = 8, 2
    a = torch.full((1, nc * m, nc * m), 2.5, dtype=torch.float64, device="cuda")
    So = sm.upscale(a, nc, nc, m, bc=sm.BC_OSCILLATORY)
    Sl = sm.upscale(a, nc, nc, m)
    torch.cuda.synchronize()
    assert (So - Sl).abs().max().item() < 1e-13 * Sl.abs().max().item()
    lay = W.uniform_array((nc * m,), 0.1, 10.0, 3101)
    a_np = np.tile(lay[None, :], (nc * m, 1))[None]
    S_ref, _, _ = orc.upscale(a_np, nc, nc, m, bc=orc.BC_OSC)
    Sg = sm.upscale(torch.from_numpy(np.ascontiguousarray(a_np)).cuda(), nc, nc, m, bc=sm.BC_OSCILLATORY)
    torch.cuda.synchronize()
    Sg = Sg.cpu().numpy()
    assert (np.abs(Sg - S_ref).max(-1) / np.abs(S_ref).max(-1)).max() < 1e-10


def test_oscillatory_boundary_data_rejects_refinement(sm):
    a = torch.ones((1, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(sm.StomsfemError) as e:
        sm.upscale(a, 1, 1, 8, precision=sm.PREC_F32_REFINE64, bc=sm.BC_OSCILLATORY)
    assert e.value.code == sm.EINVAL
    with pytest.raises(sm.StomsfemError) as e:
        sm.upscale(a, 1, 1, 8, bc=7)
    assert e.value.code == sm.EINVAL
