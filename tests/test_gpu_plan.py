"""Execution plans (graph-captured stages of mixed H/h): every replay of the
whole plan and of single stages equals the eager path, and the eager path
equals the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem
    return stomsfem


def _eager(sm, st, fam_kw, xi, nc, m, a_dtype):
    if "bumps" in fam_kw:
        a = sm.coef_bumps(xi, nc * m, **fam_kw["params"], dtype=a_dtype)
    else:
        a = sm.coef_features(fam_kw["feature_map"], fam_kw["nfeat"], xi, fam_kw["decades"], dtype=a_dtype)
    S = sm.upscale(a, nc, nc, m)
    return sm.coarse_solve(S, nc, nc)


def test_plan_replays_equal_eager_path(sm):
    dev = "cuda"
    wl8 = W.MESH8
    bump_params = wl8.coef_params()
    fam = sm.bump_family(wl8)
    ch = W.CHANNELS64
    kind, x0, y0, size = W.channel_geometry(ch)
    g = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in (kind, x0, y0, size)]
    nc_ch = 16  # a smaller mesh of the same medium keeps the test quick
    fmaps = {m: sm.feature_map(nc_ch * m, *g) for m in (8, 16)}
    specs = [  # (nc, m, N, family, a_dtype, seed)
        (8, 8, 64, "bumps", torch.float64, 11),
        (8, 16, 40, "bumps", torch.float64, 12),
        (nc_ch, 8, 48, "features", torch.float32, 13),
        (8, 8, 70, "bumps", torch.float32, 14),
        (nc_ch, 16, 20, "features", torch.float64, 15),
        (8, 32, 6, "bumps", torch.float64, 16),
    ]
    stages, outs, eager = [], [], []
    for nc, m, N, famname, dt, seed in specs:
        if famname == "bumps":
            xi = torch.from_numpy(W.uniform_xi(N, wl8.nxi, seed)).to(dev)
            kw = {"bumps": fam, "params": bump_params}
        else:
            xi = torch.from_numpy(W.normal_xi(N, ch.nxi, seed)).to(dev)
            kw = {"feature_map": fmaps[m], "nfeat": ch.nxi, "decades": ch.decades}
        nU = (nc - 1) ** 2
        U = torch.full((N, nU), np.nan, dtype=torch.float64, device=dev)
        qm = torch.full((nU,), np.nan, dtype=torch.float64, device=dev)
        qv = torch.full((nU,), np.nan, dtype=torch.float64, device=dev)
        st = torch.full((N, nc * nc), -9, dtype=torch.int32, device=dev)
        stages.append(sm.make_stage(nc, m, xi, bumps=kw.get("bumps"), feature_map=kw.get("feature_map"),
                                    nfeat=kw.get("nfeat", 0), decades=kw.get("decades", 4.0), a_dtype=dt,
                                    U=U, qoi_mean=qm, qoi_var=qv, status=st))
        outs.append((U, qm, qv, st, xi))
        eager.append([t.cpu().numpy() for t in _eager(sm, st, kw, xi, nc, m, dt)])
    plan = sm.plan_create(stages)
    for rep in range(3):
        for U, qm, qv, st, _ in outs:
            U.fill_(np.nan), qm.fill_(np.nan), qv.fill_(np.nan), st.fill_(-9)
        torch.cuda.synchronize()
        if rep < 2:
            plan.launch()
        else:
            for i in range(len(stages)):
                plan.launch(i)
        torch.cuda.synchronize()
        for (U, qm, qv, st, _), (Ue, qme, qve) in zip(outs, eager):
            np.testing.assert_array_equal(U.cpu().numpy(), Ue)
            np.testing.assert_array_equal(qm.cpu().numpy(), qme)
            np.testing.assert_array_equal(qv.cpu().numpy(), qve)
            assert int((st != 0).sum()) == 0
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device=dev)
        (x * x).sum().item()
    # the eager path against the oracle on the first stage
    U0, qm0 = eager[0][0], eager[0][1]
    a = oracle.coef_bumps(outs[0][4].cpu().numpy(), wl8.nfine, **bump_params)
    Sr, _, _ = oracle.upscale(a, wl8.nc, wl8.nc, wl8.m)
    Ur, mr, _ = oracle.coarse_solve(Sr, wl8.nc, wl8.nc)
    np.testing.assert_allclose(qm0, mr, rtol=1e-10, atol=0)
    plan.free()


def test_plan_rejects_bad_stages(sm):
    xi = torch.zeros((4, 16), dtype=torch.float64, device="cuda")
    fam = sm.bump_family(W.MESH8)
    for nc, m in ((1, 8), (8, 0), (8, 49)):
        with pytest.raises(sm.StomsfemError) as e:
            sm.plan_create([sm.make_stage(nc, m, xi, bumps=fam)])
        assert e.value.code == sm.EINVAL
    with pytest.raises(sm.StomsfemError):
        sm.plan_create([])
