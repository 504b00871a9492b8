"""GPU learned surrogate of the channels-and-inclusions medium (64 x 64 coarse
mesh, 40 channels + 40 squares, conductivities 10^(4 sigmoid(xi_j)), xi_j ~
N(0,1)) through the C-ABI, against the FP64 oracle.

Every oracle input here comes from the seeded generators or from the oracle
itself: the feature map, the coefficient blocks and the training S are the
oracle's; the raw network outputs handed to the gate are built from the
oracle's S.  Tolerances: the standardisation within 1e-13 of the oracle's
(FP64 on both sides, different summation orders); the FP32 forward pass of
the untrained network within 1e-5 (absolute, standardised units) of the FP64
oracle's on the same FP32-rounded inputs, the BF16 pass within 1e-3; the gate
on identical raw outputs: accept mask exact, residual and uncertainty within
1e-12 relative, stored S within 1e-10 relative to max|S| of the pair.  The
end-to-end criterion is the coarse solution: surrogate within 1e-3 (relative,
per sample) of the plain FP64 path, and of the oracle on sampled whole
samples; recomputed pairs equal the plain path's bit for bit.
"""
import numpy as np
import pytest
import torch

from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu

WL = W.CHANNELS64


def say(msg):
    print(f"[gpu-mlp-features] {msg}", flush=True)


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem

    stomsfem.lib()
    return stomsfem


def _oracle_map(orc, nf):
    # the oracle's own feature map: with pairwise distinct conductivities the
    # owner of every fine element is read off the oracle's coefficient
    kind, x0, y0, size = W.channel_geometry(WL)
    xi_id = np.linspace(-2.0, 2.0, WL.nxi)[None, :]
    a_id = orc.coef_features(xi_id, nf, kind, x0, y0, size, decades=WL.decades)[0]
    th = 10.0 ** (WL.decades / (1.0 + np.exp(-xi_id[0])))
    assert len(np.unique(th)) == WL.nxi
    assert np.diff(np.sort(th)).min() > 1e-6 * th.max() and th.min() > 2.0
    fmap = np.full((nf, nf), -1, dtype=np.int32)
    for j in range(WL.nxi):   # (libm and numpy may differ in the last bit)
        fmap[np.abs(a_id - th[j]) <= 1e-12 * th[j]] = j
    assert (fmap[a_id != 1.0] >= 0).all()
    return fmap


def _blocks(a, nc, m):
    # [N][nc*m][nc*m] -> [N][M][m][m], K = ky*nc + kx
    N = a.shape[0]
    return a.reshape(N, nc, m, nc, m).transpose(0, 1, 3, 2, 4).reshape(N, nc * nc, m, m)


@pytest.fixture(scope="module")
def small(sm, orc):
    # H/h = 8, 16 training samples from the oracle, untrained network
    from oracle import mlp
    m, nc = 8, WL.nc
    nf = nc * m
    kind, x0, y0, size = W.channel_geometry(WL)
    dev = [torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in (kind, x0, y0, size)]
    fmap_d = sm.feature_map(nf, *dev)
    fmap = _oracle_map(orc, nf)
    xi = W.normal_xi(16, WL.nxi, 7105)
    xi[3, :] = 3.5          # every variable outside the box [-3, 3]
    a = orc.coef_features(xi, nf, kind, x0, y0, size, decades=WL.decades)
    S, st, _ = orc.upscale(a, nc, nc, m)
    assert (st == 0).all()
    lf = mlp.local_features(fmap, nc, nc, m)
    init = W.mlp_init(WL.M, 7005)
    model = sm.mlp_create_features(nc, m, fmap_d, WL.nxi, WL.decades, init, 3.0)
    blk = _blocks(a, nc, m)
    ring = np.array([[mlp.ring_mean(blk[s, K]) for K in range(WL.M)] for s in range(len(xi))])
    sm.mlp_set_data(model, torch.from_numpy(xi).cuda(), torch.from_numpy(np.ascontiguousarray(S)).cuda())
    say(f"small model: local features per patch {np.bincount([len(f) for f in lf]).tolist()}")
    yield dict(m=m, fmap_d=fmap_d, fmap=fmap, xi=xi, S=S, lf=lf, init=init, model=model, ring=ring)
    model.free()


def test_feature_map_and_local_variables(sm, small):
    np.testing.assert_array_equal(small["fmap_d"].cpu().numpy(), small["fmap"])
    lv, nl = sm.local_vars_features(WL.nc, WL.nc, small["m"], small["fmap"], WL.nxi)
    for K, f in enumerate(small["lf"]):
        assert nl[K] == len(f)
        assert lv[K].tolist() == (f + [-1] * (4 - len(f)) if len(f) <= 4 else [-2, -1, -1, -1])
    assert (nl == 0).sum() > 0 and (nl >= 2).sum() > 0


def test_standardization_matches_oracle(sm, small):
    # targets S_K / (mean conductivity on K's boundary ring)
    from oracle import mlp
    xi, S, ring = small["xi"], small["S"], small["ring"]
    mu, sd = sm.mlp_standardization(small["model"])
    for K in range(WL.M):
        mu_o, sd_o = mlp.standardize(S[:, K] / ring[:, K, None])
        tol = 1e-13 * max(1.0, np.abs(mu_o).max())
        assert np.abs(mu[K] - mu_o).max() <= tol, K
        assert np.abs(sd[K] - sd_o).max() <= tol, K
    say(f"standardisation agrees on {WL.M} patches")


def test_forward_transformed_inputs_match_oracle(sm, small):
    # the untrained network (seeded initial weights) on u_j = 2 sigmoid(xi_j) - 1
    from oracle import mlp
    xi, lf, init, model = small["xi"], small["lf"], small["init"], small["model"]
    xi_d = torch.from_numpy(xi).cuda()
    Y32 = sm.mlp_predict(model, xi_d, sm.PREC_F32).cpu().numpy()
    Y16 = sm.mlp_predict(model, xi_d, sm.PREC_BF16).cpu().numpy()
    w32 = w16 = 0.0
    for K in range(WL.M):
        X = np.zeros((len(xi), 4))
        if len(lf[K]) <= 4:
            X[:, :len(lf[K])] = mlp.features_input(xi[:, lf[K]])
        X = X.astype(np.float32).astype(np.float64)
        Yref, _ = mlp.forward(init[K].astype(np.float64), X, 4)
        sc = max(1.0, np.abs(Yref).max())
        w32 = max(w32, float(np.abs(Y32[:, K] - Yref).max() / sc))
        w16 = max(w16, float(np.abs(Y16[:, K] - Yref).max() / sc))
    say(f"forward: FP32 {w32:.2e}, BF16 {w16:.2e} against the oracle")
    assert w32 < 1e-5 and w16 < 1e-3


def test_gate_matches_oracle(sm, small):
    # raw outputs built from the oracle's S: exact heads, seeded noise of
    # three sizes, planted NaN / inf / head disagreement; the out-of-box
    # sample and the patches with more than four features never pass
    from oracle import mlp
    xi, S, ring, lf, model = small["xi"], small["S"], small["ring"], small["lf"], small["model"]
    N = len(xi)
    mu = np.zeros((WL.M, 10))
    sd = np.zeros((WL.M, 10))
    for K in range(WL.M):
        mu[K], sd[K] = mlp.standardize(S[:, K] / ring[:, K, None])
    T = (S / ring[:, :, None] - mu[None]) / sd[None]
    Y = np.concatenate([T, T], axis=-1)
    noise = W.uniform_array(Y.shape, -1.0, 1.0, 7205)
    lvl = np.array([0.0, 1e-7, 1e-5, 1e-3])[np.arange(N) % 4]
    Y = Y + lvl[:, None, None] * noise
    Y[5, :, 2] = np.nan
    Y[6, :, 13] = np.inf
    Y[7, :, 19] += 0.5
    Y = Y.astype(np.float32)
    xi_d = torch.from_numpy(xi).cuda()
    S_g, st_g, gate_g = sm.mlp_gate(model, torch.from_numpy(Y).cuda(), xi_d, 1e-3)
    torch.cuda.synchronize()
    S_g, st_g, gate_g = S_g.cpu().numpy(), st_g.cpu().numpy(), gate_g.cpu().numpy()
    nacc = 0
    for K in range(WL.M):
        k = len(lf[K])
        X = np.zeros((N, 4))
        if k <= 4:
            X[:, :k] = xi[:, lf[K]]
        ok, Sp, resid, unc = mlp.gate(Y[:, K].astype(np.float64), mu[K], sd[K], X, min(k, 4), 1e-3, box=3.0,
                                      scale=ring[:, K])
        if k > 4:
            ok = np.zeros_like(ok)
        np.testing.assert_array_equal(st_g[:, K] == 0, ok, err_msg=f"patch {K}")
        for got, ref in ((gate_g[:, K, 0], resid), (gate_g[:, K, 1], unc)):
            assert np.array_equal(np.isnan(got), np.isnan(ref)), K
            f = ~np.isnan(ref)
            assert np.all(np.abs(got[f] - ref[f]) <= 1e-12 * np.maximum(1.0, np.abs(ref[f]))), K
        if ok.any():
            sc = np.abs(Sp[ok]).max(-1)
            assert (np.abs(S_g[ok, K] - Sp[ok]).max(-1) <= 1e-10 * sc).all(), K
        nacc += int(ok.sum())
    assert not (st_g[[5, 6]] == 0).any()
    # out of the box, or heads half a standard deviation apart: rejected
    # wherever the patch has a local variable
    has = np.array([len(f) >= 1 for f in lf])
    assert not (st_g[3][has] == 0).any() and not (st_g[7][has] == 0).any()
    assert (st_g[0] == 0).mean() > 0.9
    say(f"gate agrees on all {N * WL.M} pairs ({nacc} accepted)")


def test_features_model_is_not_saved(sm, small, tmp_path):
    with pytest.raises(sm.StomsfemError) as e:
        small["model"].save(str(tmp_path / "features.model"))
    assert e.value.code == sm.EINVAL


def test_surrogate_end_to_end_mesh16(sm, orc):
    # H/h = 16: 1024 plain training samples, 24000 Adam steps, then 256 test
    # samples through the gate with the plain fallback
    m, nc = 16, WL.nc
    nf = nc * m
    kind, x0, y0, size = W.channel_geometry(WL)
    dev = [torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in (kind, x0, y0, size)]
    fmap = sm.feature_map(nf, *dev)
    ntr = 1024
    xi_tr = torch.from_numpy(W.normal_xi(ntr, WL.nxi, 7305)).cuda()
    S_tr = torch.empty((ntr, WL.M, 10), dtype=torch.float64, device="cuda")
    for c0 in range(0, ntr, 256):
        a = sm.coef_features(fmap, WL.nxi, xi_tr[c0:c0 + 256], WL.decades)
        sm.upscale(a, nc, nc, m, S=S_tr[c0:c0 + 256])
        del a
    model = sm.mlp_create_features(nc, m, fmap, WL.nxi, WL.decades, W.mlp_init(WL.M, 7405), 3.0)
    sm.mlp_set_data(model, xi_tr, S_tr)
    perm = torch.from_numpy(W.permutation(ntr, 7505)).cuda()
    for steps, lr in ((8000, 2e-3), (8000, 5e-4), (8000, 1e-4)):
        sm.mlp_train(model, steps, lr, perm)
    say("trained the H/h = 16 model")
    N = 256
    xi_np = W.normal_xi(N, WL.nxi, 7605)
    xi = torch.from_numpy(xi_np).cuda()
    S_plain = sm.upscale(sm.coef_features(fmap, WL.nxi, xi, WL.decades), nc, nc, m)
    status = torch.full((N, WL.M), -9, dtype=torch.int32, device="cuda")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    S_sur = sm.upscale_surrogate(model, xi, 1e-3, sm.PREC_BF16, status=status, stats=stats)
    U_p, _, _ = sm.coarse_solve(S_plain, nc, nc)
    U_s, _, _ = sm.coarse_solve(S_sur, nc, nc)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    Sp, Ss = S_plain.cpu().numpy(), S_sur.cpu().numpy()
    assert set(np.unique(st)) <= {0, 1, 2}
    rec = st != 0
    assert np.array_equal(Ss[rec], Sp[rec])
    ue = (torch.linalg.norm(U_s - U_p, dim=1) / torch.linalg.norm(U_p, dim=1)).cpu().numpy()
    acc = st == 0
    say(f"accepted {acc.mean():.4f}, fallback {(st == 1).mean():.4f}, audited {(st == 2).mean():.4f}; "
        f"max U err vs plain {ue.max():.2e}")
    assert ue.max() < 1e-3
    assert acc.mean() > 0.9
    # whole samples against the oracle (coefficient, upscaling and coarse solve)
    pick = [0, N - 1]
    a_ref = orc.coef_features(xi_np[pick], nf, kind, x0, y0, size, decades=WL.decades)
    S_ref, _, _ = orc.upscale(a_ref, nc, nc, m)
    U_ref, _, _ = orc.coarse_solve(S_ref, nc, nc)
    Us = U_s.cpu().numpy()[pick]
    ue_o = np.linalg.norm(Us - U_ref, axis=1) / np.linalg.norm(U_ref, axis=1)
    r = rec[pick]
    d = np.abs(Ss[pick][r] - S_ref[r]).max(-1) / np.abs(S_ref[r]).max(-1)
    say(f"samples {pick}: max U err vs oracle {ue_o.max():.2e}, recomputed pairs {int(r.sum())} "
        f"max S diff {d.max() if d.size else 0:.1e}")
    assert ue_o.max() < 1e-3 and (d.size == 0 or d.max() < 1e-10)
    model.free()
