"""GPU reduced basis on oversampled patches (stomsfem_reduce_os /
stomsfem_reduce_os_apply, through the C-ABI) against the oracle
(oracle.rb.rb_os_online_S16 on the oracle's own patch models) and against
the GPU's plain oversampled solve.

Tolerances: the FP32 matrix-core online stage (FP32 GEMM with FP32
accumulation over the patch's Mp^2 elements, FP64 solve and recombination)
stays within 2e-4 relative per pair of the FP64 stage and of the oracle; the
FP64 online stage reproduces the oracle's S16 to 1e-7 relative per pair
(both sides build the same energy-KL subspace from the same snapshots; their
eigen-solvers differ, so agreement is bounded by the spectral gap after the
last kept mode, not by rounding); where the reduced
space holds the patch solutions exactly (a training sample with every mode
kept, or a patch with fewer interior unknowns than modes) S16 equals the
oversampled solve to 1e-9.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-rb-os] {msg}", flush=True)


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem

    stomsfem.lib()
    return stomsfem


def _bumps(orc, N, seed, nc, m):
    wl = W.MESH8
    xi = W.uniform_xi(N, wl.nxi, seed)
    return orc.coef_bumps(xi, wl.nfine, **wl.coef_params())[:, : nc * m, : nc * m].copy()


def _rel_pairs(S, R):
    """max over pairs of max_q |S_q - R_q| / max_q |R_q|."""
    S = S.reshape(S.shape[0], S.shape[1], -1)
    R = R.reshape(R.shape[0], R.shape[1], -1)
    return (np.abs(S - R).max(-1) / np.abs(R).max(-1)).max()


@pytest.fixture(scope="module")
def setup(sm, orc):
    from oracle import rb

    nc, m, o, ntr = 4, 8, 4, 24   # lower-left 4x4 elements of the 8x8 bump medium, ratio 2
    a_tr = _bumps(orc, ntr, 2103, nc, m)
    say(f"build: nc={nc} m={m} o={o} ntrain={ntr}")
    model = sm.reduce_os(torch.from_numpy(a_tr).cuda(), nc, nc, m, o, r_max=8, tail_tol=1e-6)
    orc_models = []
    for K in range(nc * nc):
        blocks = np.stack([rb.patch_block(a_tr[s], K, nc, nc, m, o) for s in range(ntr)])
        orc_models.append(rb.rb_offline(np.ascontiguousarray(blocks), r_max=8, tail_tol=1e-6))
    return dict(nc=nc, m=m, o=o, model=model, orc_models=orc_models, a_tr=a_tr)


def _oracle_S16(orc, models, a, nc, m, o):
    from oracle import rb
    out = np.zeros((a.shape[0], nc * nc, 16))
    for K in range(nc * nc):
        kx, ky = K % nc, K // nc
        cx = kx * m - orc.os_origin(kx, m, o, nc * m)
        cy = ky * m - orc.os_origin(ky, m, o, nc * m)
        for s in range(a.shape[0]):
            blk = np.ascontiguousarray(rb.patch_block(a[s], K, nc, nc, m, o))
            out[s, K] = rb.rb_os_online_S16(models[K], blk, m, cx, cy).ravel()
    return out


def test_r_per_patch_matches_oracle(sm, setup):
    r = np.zeros(setup["nc"] ** 2, dtype=np.int32)
    sm.lib().stomsfem_model_export(setup["model"].handle, 0, r.ctypes.data, r.nbytes)
    assert list(r) == [mo["r"] for mo in setup["orc_models"]]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_online_matches_oracle(sm, orc, setup, dtype):
    nc, m, o = setup["nc"], setup["m"], setup["o"]
    a = _bumps(orc, 5, 1103, nc, m).astype(dtype)
    say(f"online vs oracle, dtype={np.dtype(dtype).name}")
    st = torch.full((5, nc * nc), 99, dtype=torch.int32, device="cuda")
    S = sm.reduce_os_apply(setup["model"], torch.from_numpy(a).cuda(), status=st).cpu().numpy()
    assert (st == sm.OK).all()
    R = _oracle_S16(orc, setup["orc_models"], a.astype(np.float64), nc, m, o)
    err = _rel_pairs(S, R)
    say(f"max rel err {err:.2e}")
    assert err < 1e-7


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_matrix_core_stage_matches_oracle_and_fp64(sm, orc, setup, dtype):
    # 130 samples: one full tile of 128 samples per patch and a ragged one
    nc, m, o = setup["nc"], setup["m"], setup["o"]
    a_np = _bumps(orc, 130, 1107, nc, m).astype(dtype)
    a = torch.from_numpy(a_np).cuda()
    say(f"FP32 matrix-core stage, dtype={np.dtype(dtype).name}")
    st = torch.full((130, nc * nc), 99, dtype=torch.int32, device="cuda")
    S32 = sm.reduce_os_apply(setup["model"], a, status=st, precision=sm.PREC_F32).cpu().numpy()
    assert (st == sm.OK).all()
    S64 = sm.reduce_os_apply(setup["model"], a).cpu().numpy()
    err = _rel_pairs(S32, S64)
    say(f"vs FP64 stage: {err:.2e}")
    assert err < 2e-4
    idx = [0, 1, 127, 128, 129]
    R = _oracle_S16(orc, setup["orc_models"], a_np[idx].astype(np.float64), nc, m, o)
    assert _rel_pairs(S32[idx], R) < 2e-4


@pytest.mark.parametrize("m,o,nc", [(4, 2, 5), (8, 2, 3), (6, 3, 3), (16, 8, 2)])
def test_matrix_core_stage_patch_shapes(sm, orc, m, o, nc):
    # patch sides 8 (rows not on 16-byte boundaries: scalar loads), 12 and 12
    # (neither 8, 16 nor 32), 32 (vector loads); FP32 coefficients
    a_tr = torch.from_numpy(_bumps(orc, 12, 2107, nc, m)).cuda()
    a = torch.from_numpy(_bumps(orc, 7, 2108, nc, m).astype(np.float32)).cuda()
    say(f"matrix-core stage m={m} o={o} nc={nc}")
    model = sm.reduce_os(a_tr, nc, nc, m, o, r_max=8, tail_tol=1e-6)
    st = torch.full((7, nc * nc), 99, dtype=torch.int32, device="cuda")
    S32 = sm.reduce_os_apply(model, a, status=st, precision=sm.PREC_F32).cpu().numpy()
    assert (st == sm.OK).all()
    S64 = sm.reduce_os_apply(model, a).cpu().numpy()
    assert _rel_pairs(S32, S64) < 2e-4


def test_ragged_sample_blocks(sm, orc, setup):
    # 70 samples: one full wavefront of samples per patch and a ragged one;
    # every pair equals the same pair computed alone
    nc, m = setup["nc"], setup["m"]
    a = torch.from_numpy(_bumps(orc, 70, 1104, nc, m)).cuda()
    say("ragged sample blocks")
    S = sm.reduce_os_apply(setup["model"], a)
    for s in (0, 63, 64, 69):
        S1 = sm.reduce_os_apply(setup["model"], a[s:s + 1].contiguous())
        assert torch.equal(S[s:s + 1], S1), s
    assert torch.isfinite(S).all()


@pytest.mark.parametrize("ntr,r_expect", [(1, 0), (2, 3), (3, 6)])
def test_training_samples_reproduce_the_oversampled_solve(sm, orc, ntr, r_expect):
    # ntr training samples: their centred snapshots span 3 (ntr - 1)
    # directions (the numerical rank; r = 0 for one sample, psi = phibar),
    # all kept, so each training sample's patch solutions lie in the reduced
    # space
    nc, m, o = 4, 8, 4
    a = torch.from_numpy(_bumps(orc, ntr, 2104, nc, m)).cuda()
    say(f"training samples vs upscale_os, ntrain={ntr}")
    model = sm.reduce_os(a, nc, nc, m, o, r_max=8, tail_tol=0.0)
    r = np.zeros(nc * nc, dtype=np.int32)
    sm.lib().stomsfem_model_export(model.handle, 0, r.ctypes.data, r.nbytes)
    assert (r == r_expect).all()
    S = sm.reduce_os_apply(model, a)
    R = sm.upscale_os(a, nc, nc, m, o)
    err = _rel_pairs(S.cpu().numpy(), R.cpu().numpy())
    say(f"max rel err {err:.2e}")
    assert err < 1e-9


@pytest.mark.parametrize("m,o,nc", [(2, 0, 3), (3, 0, 2), (1, 1, 3)])
def test_tiny_patches_are_exact(sm, orc, m, o, nc):
    # patches of 2 or 3 cells: at most 4 interior unknowns, fewer than the
    # modes, so the reduced space is the whole space for any sample
    a_tr = torch.from_numpy(W.uniform_array((6, nc * m, nc * m), 0.3, 4.0, 2105)).cuda()
    a = torch.from_numpy(W.uniform_array((3, nc * m, nc * m), 0.3, 4.0, 2106)).cuda()
    say(f"tiny patches m={m} o={o} nc={nc}")
    model = sm.reduce_os(a_tr, nc, nc, m, o, r_max=8, tail_tol=0.0)
    S = sm.reduce_os_apply(model, a)
    R = sm.upscale_os(a, nc, nc, m, o)
    assert _rel_pairs(S.cpu().numpy(), R.cpu().numpy()) < 1e-9


def test_bad_coefficient_flags_the_patches_that_hold_it(sm, orc, setup):
    nc, m, o = setup["nc"], setup["m"], setup["o"]
    a_np = _bumps(orc, 2, 1105, nc, m)
    a_np[1, 13, 2] = np.nan
    say("NaN coefficient")
    st = torch.full((2, nc * nc), 99, dtype=torch.int32, device="cuda")
    sm.reduce_os_apply(setup["model"], torch.from_numpy(a_np).cuda(), status=st)
    st = st.cpu().numpy()
    assert (st[0] == sm.OK).all()
    for K in range(nc * nc):
        kx, ky = K % nc, K // nc
        x0, y0 = orc.os_origin(kx, m, o, nc * m), orc.os_origin(ky, m, o, nc * m)
        holds = x0 <= 2 < x0 + m + 2 * o and y0 <= 13 < y0 + m + 2 * o
        assert st[1, K] == (sm.ENOTSPD if holds else sm.OK), K


def test_invalid_arguments(sm, orc, setup):
    nc, m = setup["nc"], setup["m"]
    a = torch.from_numpy(_bumps(orc, 2, 1106, nc, m)).cuda()
    say("invalid arguments")
    with pytest.raises(sm.StomsfemError) as e:   # patch of 34 cells
        sm.reduce_os(a, nc, nc, m, 13)
    assert e.value.code == sm.EINVAL
    with pytest.raises(sm.StomsfemError) as e:   # patch wider than the 2-element domain
        sm.reduce_os(a[:, :16, :16].contiguous(), 2, 2, m, 8)
    assert e.value.code == sm.EINVAL
    with pytest.raises(sm.StomsfemError) as e:
        sm.reduce_os_apply(setup["model"], a, precision=sm.PREC_BF16)
    assert e.value.code == sm.EINVAL
    with pytest.raises(sm.StomsfemError) as e:   # the oversampled model is not a plain one
        sm.reduce_apply(setup["model"], a, precision=sm.PREC_F64)
    assert e.value.code == sm.EINVAL
    plain = sm.reduce(a, nc, nc, m, r_max=4)
    with pytest.raises(sm.StomsfemError) as e:
        sm.reduce_os_apply(plain, a)
    assert e.value.code == sm.EINVAL
    # batch mesh differs from the model's (m = 4 on the same 32 x 32 grid)
    a4 = a[:, :4 * 4, :4 * 4].contiguous()
    S4 = torch.empty((2, nc * nc, 16), dtype=torch.float64, device="cuda")
    b = sm.Batch(nc, nc, 4, sm.F64, 2, a4.data_ptr(), S4.data_ptr(), None)
    assert sm.lib().stomsfem_reduce_os_apply(setup["model"].handle, ctypes.byref(b), sm.PREC_F64, None) == sm.EINVAL
    # empty batch
    S = sm.reduce_os_apply(setup["model"], a[:0])
    assert S.shape == (0, nc * nc, 16)


def test_full_size_sampled_against_oracle(sm, orc):
    # the benchmark's launch: the 8x8 bump mesh, ratio 2, 64 training
    # samples (seed 2003), 16 384 online samples in FP32 through the
    # matrix-core stage; 24 sampled pairs against the oracle's own patch
    # models (each built from the same training fields)
    from oracle import rb

    wl = W.MESH8
    nc, m, o, ntr, N = wl.nc, wl.m, 4, 64, 16384
    xi_tr = W.uniform_xi(ntr, wl.nxi, 2003)
    a_tr = orc.coef_bumps(xi_tr, wl.nfine, **wl.coef_params())
    xi = torch.from_numpy(W.uniform_xi(N, wl.nxi, wl.seed)).cuda()
    say("full size: build")
    model = sm.reduce_os(torch.from_numpy(a_tr).cuda(), nc, nc, m, o, r_max=8, tail_tol=1e-6)
    a32 = sm.coef_bumps(xi, wl.nfine, **wl.coef_params(), dtype=torch.float32)
    st = torch.full((N, wl.M), 99, dtype=torch.int32, device="cuda")
    say("full size: online")
    S = sm.reduce_os_apply(model, a32, status=st, precision=sm.PREC_F32).cpu().numpy()
    assert (st == sm.OK).all()
    rng = np.random.default_rng(77)
    samples = rng.integers(0, N, size=24)
    patches = rng.integers(0, wl.M, size=24)
    samples[:2] = (0, N - 1)
    a_s = a32[torch.from_numpy(samples).cuda()].double().cpu().numpy()
    models = {}
    worst = 0.0
    for i, (s, K) in enumerate(zip(samples, patches)):
        K = int(K)
        if K not in models:
            blocks = np.stack([rb.patch_block(a_tr[t], K, nc, nc, m, o) for t in range(ntr)])
            models[K] = rb.rb_offline(np.ascontiguousarray(blocks), r_max=8, tail_tol=1e-6)
        kx, ky = K % nc, K // nc
        cx = kx * m - orc.os_origin(kx, m, o, nc * m)
        cy = ky * m - orc.os_origin(ky, m, o, nc * m)
        R = rb.rb_os_online_S16(models[K], np.ascontiguousarray(rb.patch_block(a_s[i], K, nc, nc, m, o)), m, cx, cy)
        worst = max(worst, np.abs(S[s, K] - R.ravel()).max() / np.abs(R).max())
    say(f"full size: worst sampled rel err {worst:.2e}")
    assert worst < 2e-4


def test_high_contrast_patches_of_24_cells(sm, orc):
    # two-phase medium (1 or 1e4 per fine cell), patches of 24 cells (ratio
    # 3): the FP64 snapshots of the build (band in 123 KB of LDS) and the
    # exact reproduction of the training samples (r = 3 for two samples)
    nc, m, o = 3, 8, 8
    rng = np.random.default_rng(2109)
    a_np = np.where(rng.random((2, nc * m, nc * m)) < 0.3, 1e4, 1.0)
    a = torch.from_numpy(a_np).cuda()
    say("high-contrast patches of 24 cells")
    model = sm.reduce_os(a, nc, nc, m, o, r_max=8, tail_tol=0.0)
    r = np.zeros(nc * nc, dtype=np.int32)
    sm.lib().stomsfem_model_export(model.handle, 0, r.ctypes.data, r.nbytes)
    assert (r == 3).all()
    S = sm.reduce_os_apply(model, a).cpu().numpy()
    R, _ = orc.upscale_os(a_np, nc, nc, m, o)
    assert _rel_pairs(S, R) < 1e-8


@pytest.mark.parametrize("m,o,nc", [(8, 16, 5), (20, 20, 3), (32, 16, 2)])
def test_patches_beyond_32_cells_reproduce_training_samples(sm, m, o, nc):
    # patches of 40, 60 (Sec. 5.2: H/h = 20, ratio 3) and 64 cells (the Sec.
    # 5.3 mesh's): snapshots from the band-window kernel; two training
    # samples (r = 3) are reproduced exactly, so S16 equals the oversampled
    # solve of those samples; the FP32 matrix-core stage within 2e-4
    a = torch.from_numpy(W.uniform_array((2, nc * m, nc * m), 0.3, 4.0, 2110 + m)).cuda()
    say(f"patch of {m + 2 * o} cells: build")
    model = sm.reduce_os(a, nc, nc, m, o, r_max=8, tail_tol=0.0)
    r = np.zeros(nc * nc, dtype=np.int32)
    sm.lib().stomsfem_model_export(model.handle, 0, r.ctypes.data, r.nbytes)
    assert (r == 3).all()
    S = sm.reduce_os_apply(model, a)
    R = sm.upscale_os(a, nc, nc, m, o)
    err = _rel_pairs(S.cpu().numpy(), R.cpu().numpy())
    say(f"  vs oversampled solve {err:.2e}")
    assert err < 1e-8
    S32 = sm.reduce_os_apply(model, a.float(), precision=sm.PREC_F32)
    assert _rel_pairs(S32.cpu().numpy(), S.cpu().numpy()) < 2e-4


def test_40_cell_patches_match_oracle(sm, orc):
    # the band-window snapshots, the dual build and both online stages at 40
    # cells against the oracle's own patch models on three patches (corner,
    # centre, corner); three training samples keep every mode (r = 6)
    from oracle import rb
    nc, m, o = 5, 8, 16
    a_tr = W.uniform_array((3, nc * m, nc * m), 0.3, 4.0, 2120)
    a = W.uniform_array((2, nc * m, nc * m), 0.3, 4.0, 2121)
    say("40-cell patches against the oracle")
    model = sm.reduce_os(torch.from_numpy(a_tr).cuda(), nc, nc, m, o, r_max=8, tail_tol=0.0)
    S = sm.reduce_os_apply(model, torch.from_numpy(a).cuda()).cpu().numpy()
    for K in (0, 12, 24):
        blocks = np.stack([rb.patch_block(a_tr[s], K, nc, nc, m, o) for s in range(3)])
        mo = rb.rb_offline(np.ascontiguousarray(blocks), r_max=8, tail_tol=0.0)
        assert mo["r"] == 6
        kx, ky = K % nc, K // nc
        cx = kx * m - orc.os_origin(kx, m, o, nc * m)
        cy = ky * m - orc.os_origin(ky, m, o, nc * m)
        for s in range(2):
            R = rb.rb_os_online_S16(mo, np.ascontiguousarray(rb.patch_block(a[s], K, nc, nc, m, o)), m, cx, cy)
            err = np.abs(S[s, K] - R.ravel()).max() / np.abs(R).max()
            assert err < 1e-7, (K, s, err)
