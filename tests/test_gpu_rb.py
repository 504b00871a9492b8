"""GPU reduced-basis path (offline build + online stage, through the C-ABI)
against the reduced-basis oracle and the plain oracle.

Tolerances: the FP64 online stage reproduces the oracle's S_rb to 1e-7
relative (both build the same energy-KL subspace from the same snapshots;
the eigen-solvers differ, so agreement is limited by the spectral gap after
the 8th mode, not by rounding); the FP32 MFMA stage to 2e-4 relative
(single-precision GEMM with 64-term FP32 accumulation); the coarse solution
through the reduced path stays within 1e-3 of the plain path.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-rb] {msg}", flush=True)


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem

    stomsfem.lib()
    return stomsfem


@pytest.fixture(scope="module")
def setup(sm, orc):
    from oracle import rb

    wl = W.MESH8
    nc, m = 4, 8   # the lower-left 4x4 coarse elements of the 8x8 bump workload
    ntr = 24
    xi_tr = W.uniform_xi(ntr, wl.nxi, 2003)
    xi_te = W.uniform_xi(6, wl.nxi, 1003)
    a_tr = orc.coef_bumps(xi_tr, wl.nfine, **wl.coef_params())[:, : nc * m, : nc * m].copy()
    a_te = orc.coef_bumps(xi_te, wl.nfine, **wl.coef_params())[:, : nc * m, : nc * m].copy()
    say(f"build: nc={nc} m={m} ntrain={ntr}")
    model = sm.reduce(torch.from_numpy(a_tr).cuda(), nc, nc, m, r_max=8, tail_tol=1e-6)
    orc_models = []
    for K in range(nc * nc):
        kx, ky = K % nc, K // nc
        orc_models.append(rb.rb_offline(a_tr[:, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m], r_max=8, tail_tol=1e-6))
    return dict(nc=nc, m=m, model=model, orc_models=orc_models, a_te=a_te)


def _oracle_S(setup, a):
    from oracle import rb
    nc, m = setup["nc"], setup["m"]
    out = np.zeros((a.shape[0], nc * nc, 10))
    for s in range(a.shape[0]):
        for K in range(nc * nc):
            kx, ky = K % nc, K // nc
            out[s, K] = rb.rb_online_S(setup["orc_models"][K], a[s, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m])
    return out


def rel(S, R):
    return (np.abs(S - R).max(-1) / np.abs(R).max(-1)).max()


def test_rb_offline_matches_oracle(sm, setup):
    say("offline: r and eigenvalues")
    r = setup["model"].export("r")
    lam = setup["model"].export("lambda")
    for K, om in enumerate(setup["orc_models"]):
        assert r[K] == om["r"]
        ref = om["sigma"][:8] ** 2
        np.testing.assert_allclose(lam[K, :8], ref, rtol=1e-8, atol=1e-12 * ref[0])


def test_rb_online_f64_matches_oracle(sm, setup):
    say("online FP64")
    a = setup["a_te"]
    S = sm.reduce_apply(setup["model"], torch.from_numpy(a).cuda(), precision=sm.PREC_F64)
    torch.cuda.synchronize()
    assert rel(S.cpu().numpy(), _oracle_S(setup, a)) < 1e-7


def test_rb_online_mfma_fp32(sm, orc, setup):
    say("online FP32 MFMA")
    a = setup["a_te"]
    for dt in (torch.float64, torch.float32):
        st = torch.full((a.shape[0], setup["nc"] ** 2), 99, dtype=torch.int32, device="cuda")
        S = sm.reduce_apply(setup["model"], torch.from_numpy(a).to(dt).cuda(), status=st)
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == 0).all()
        assert rel(S.cpu().numpy(), _oracle_S(setup, a)) < 2e-4
    # against the plain path: the reduced-basis error itself
    S_plain, _, _ = orc.upscale(a, setup["nc"], setup["nc"], setup["m"])
    assert rel(S.cpu().numpy(), S_plain) < 1e-3


def test_rb_mfma_multi_tile_workgroups_with_a_partial_group(sm, setup):
    # at H/h = 8 a workgroup takes up to eight 128-sample tiles of its patch;
    # 515 tiles per patch (the last one ragged) leave the last workgroup of
    # each patch three tiles: every pair against the FP64 stage (2e-4)
    nc, m = setup["nc"], setup["m"]
    wl = W.MESH8
    N = 128 * 515 - 58
    say(f"multi-tile workgroups: {N} samples")
    xi = torch.from_numpy(W.uniform_xi(N, wl.nxi, 1009)).cuda()
    a32 = sm.coef_bumps(xi, wl.nfine, **wl.coef_params(), dtype=torch.float32)[:, : nc * m, : nc * m].contiguous()
    st = torch.full((N, nc * nc), 99, dtype=torch.int32, device="cuda")
    S32 = sm.reduce_apply(setup["model"], a32, status=st, precision=sm.PREC_F32)
    S64 = sm.reduce_apply(setup["model"], a32, precision=sm.PREC_F64)
    torch.cuda.synchronize()
    assert (st == sm.OK).all()
    err = ((S32 - S64).abs().amax(dim=2) / S64.abs().amax(dim=2)).max().item()
    say(f"  max rel err vs FP64 stage {err:.2e}")
    assert err < 2e-4


def test_rb_coarse_solution_error(sm, orc, setup):
    say("coarse solution through the reduced path")
    a = setup["a_te"]
    nc, m = setup["nc"], setup["m"]
    S = sm.reduce_apply(setup["model"], torch.from_numpy(a).cuda())
    U, _, _ = sm.coarse_solve(S, nc, nc)
    torch.cuda.synchronize()
    S_plain, _, _ = orc.upscale(a, nc, nc, m)
    U_plain, _, _ = orc.coarse_solve(S_plain, nc, nc)
    err = np.linalg.norm(U.cpu().numpy() - U_plain, axis=1) / np.linalg.norm(U_plain, axis=1)
    assert err.max() < 1e-3


def test_rb_full_size_against_oracle(sm, orc):
    # the reduced-basis workload at its own size: the whole 8x8 mesh, 256
    # training samples per patch (seed 2003), 16 384 online samples (seed 1003)
    # with FP32 coefficients through the FP32 MFMA stage in one launch;
    # offline r and eigenvalues of every patch against the oracle, whole
    # online samples (first, last, six seeded) against the oracle's S_rb (2e-4)
    # and the oracle's plain coarse solution (1e-3)
    from oracle import rb
    wl = W.MESH8
    nc, m = wl.nc, wl.m
    ntr, N = 256, 16384
    xi_tr = W.uniform_xi(ntr, wl.nxi, 2003)
    a_tr = orc.coef_bumps(xi_tr, wl.nfine, **wl.coef_params())
    say(f"full-size build: {nc}x{nc} mesh, m={m}, {ntr} training samples")
    model = sm.reduce(torch.from_numpy(a_tr).cuda(), nc, nc, m, r_max=8, tail_tol=1e-6)
    r = model.export("r")
    lam = model.export("lambda")
    orc_models = []
    for K in range(nc * nc):
        kx, ky = K % nc, K // nc
        om = rb.rb_offline(a_tr[:, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m], r_max=8, tail_tol=1e-6)
        assert r[K] == om["r"], K
        ref = om["sigma"][:8] ** 2
        np.testing.assert_allclose(lam[K, :8], ref, rtol=1e-8, atol=1e-12 * ref[0])
        orc_models.append(om)
    xi = torch.from_numpy(W.uniform_xi(N, wl.nxi, 1003)).cuda()
    a32 = sm.coef_bumps(xi, wl.nfine, **wl.coef_params(), dtype=torch.float32)
    st = torch.full((N, nc * nc), 99, dtype=torch.int32, device="cuda")
    S = sm.reduce_apply(model, a32, status=st, precision=sm.PREC_F32)
    U, _, _ = sm.coarse_solve(S, nc, nc)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    pick = np.unique(np.concatenate([[0, N - 1], np.random.default_rng(3103).choice(N, 6, replace=False)]))
    a = a32.cpu().numpy()[pick].astype(np.float64)
    Sg = S.cpu().numpy()[pick]
    S_rb = np.zeros_like(Sg)
    for i in range(len(pick)):
        for K in range(nc * nc):
            kx, ky = K % nc, K // nc
            S_rb[i, K] = rb.rb_online_S(orc_models[K], a[i, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m])
    assert rel(Sg, S_rb) < 2e-4
    S_plain, _, _ = orc.upscale(a, nc, nc, m)
    U_plain, _, _ = orc.coarse_solve(S_plain, nc, nc)
    ue = np.linalg.norm(U.cpu().numpy()[pick] - U_plain, axis=1) / np.linalg.norm(U_plain, axis=1)
    say(f"samples {pick.tolist()}: S_rb err {rel(Sg, S_rb):.2e}, U err vs plain oracle {ue.max():.2e}")
    assert ue.max() < 1e-3
    model.free()


@pytest.mark.parametrize("m,nsub,ntr,form", [(16, 2, 80, "primal"), (16, 2, 24, "dual"), (32, 2, 40, "dual")])
def test_rb_larger_cells_against_oracle(sm, orc, m, nsub, ntr, form):
    # the reduced basis at H/h = 16 and 32 on nsub x nsub interior patches of
    # the 32 x 32 bump workload's geometry (fine grid 32 m): the
    # offline build in its primal form (3 ntrain >= (m-1)^2) and in the dual
    # form (the method of snapshots, with the snapshots from the refined
    # FP32/FP64 solver at m = 32), then both online stages against the oracle
    from oracle import rb
    wl = W.MESH32
    nf = wl.nc * m
    xi_tr = W.uniform_xi(ntr, wl.nxi, 2032 + m)
    xi_te = W.uniform_xi(5, wl.nxi, 1032 + m)
    cp = wl.coef_params()
    o = 5 * m  # patches (5, 5).. of the mesh: up to four local variables each
    a_tr = orc.coef_bumps(xi_tr, nf, **cp)[:, o:o + nsub * m, o:o + nsub * m].copy()
    a_te = orc.coef_bumps(xi_te, nf, **cp)[:, o:o + nsub * m, o:o + nsub * m].copy()
    say(f"m={m}: {form} build, {ntr} training samples, {nsub}x{nsub} patches")
    model = sm.reduce(torch.from_numpy(a_tr).cuda(), nsub, nsub, m, r_max=8, tail_tol=1e-6)
    r = model.export("r")
    lam = model.export("lambda")
    oms = []
    for K in range(nsub * nsub):
        kx, ky = K % nsub, K // nsub
        om = rb.rb_offline(a_tr[:, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m], r_max=8, tail_tol=1e-6)
        assert r[K] == om["r"], K
        ref = om["sigma"][:8] ** 2
        np.testing.assert_allclose(lam[K, :8], ref, rtol=1e-8, atol=1e-12 * ref[0])
        oms.append(om)
    S_ref = np.zeros((a_te.shape[0], nsub * nsub, 10))
    for s in range(a_te.shape[0]):
        for K in range(nsub * nsub):
            kx, ky = K % nsub, K // nsub
            S_ref[s, K] = rb.rb_online_S(oms[K], a_te[s, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m])
    S64 = sm.reduce_apply(model, torch.from_numpy(a_te).cuda(), precision=sm.PREC_F64).cpu().numpy()
    st = torch.full((a_te.shape[0], nsub * nsub), 99, dtype=torch.int32, device="cuda")
    S32 = sm.reduce_apply(model, torch.from_numpy(a_te).float().cuda(), status=st, precision=sm.PREC_F32)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    e64, e32 = rel(S64, S_ref), rel(S32.cpu().numpy(), S_ref.astype(np.float64))
    S_plain, _, _ = orc.upscale(a_te, nsub, nsub, m)
    say(f"m={m} {form}: r={r.tolist()}, FP64 online vs oracle {e64:.2e}, MFMA vs oracle {e32:.2e}, "
        f"RB vs plain {rel(S64, S_plain):.2e}")
    assert e64 < 1e-7
    assert e32 < 2e-4
    model.free()


@pytest.mark.parametrize("m", [40, 48])
def test_rb_cells_beyond_32_reproduce_training_samples(sm, m):
    # H/h = 40 and 48: the band-window snapshot kernel and the method of
    # snapshots; two training samples (r = 3) are reproduced exactly, so S_rb
    # equals the plain upscaling of those samples (both online stages)
    nc = 2
    a = torch.from_numpy(W.uniform_array((2, nc * m, nc * m), 0.3, 4.0, 2130 + m)).cuda()
    say(f"H/h = {m}: build")
    model = sm.reduce(a, nc, nc, m, r_max=8, tail_tol=0.0)
    assert (model.export("r") == 3).all()
    S_ref = sm.upscale(a, nc, nc, m)
    for prec, tol in ((sm.PREC_F64, 1e-9), (sm.PREC_F32, 2e-4)):
        S = sm.reduce_apply(model, a if prec == sm.PREC_F64 else a.float(), precision=prec)
        err = rel(S.cpu().numpy(), S_ref.cpu().numpy())
        say(f"  precision {prec}: {err:.2e}")
        assert err < tol
    model.free()
