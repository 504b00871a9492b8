"""Model files: every model kind reloads with bitwise-identical online results."""
import numpy as np
import pytest
import torch

from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem
    return stomsfem


def test_interpolation_model_roundtrip(sm, tmp_path):
    wl = W.MESH8
    fam = sm.bump_family(wl)
    lv, _ = sm.local_vars_bumps(wl.nc, wl.nc, wl.m, fam)
    model = sm.interp_build(wl.nc, wl.nc, wl.m, lv, fam, 4, -0.8, 0.8)
    path = str(tmp_path / "ri.bin")
    model.save(path)
    again = sm.model_load(path)
    assert (again.ncx, again.ncy, again.m) == (wl.nc, wl.nc, wl.m)
    np.testing.assert_array_equal(again.export("table"), model.export("table"))
    xi = torch.from_numpy(W.uniform_xi(100, wl.nxi, 7101)).cuda()  # some pairs leave the box
    sm.stats_reset()
    S1, n1 = sm.interp_apply(model, xi)
    S2, n2 = sm.interp_apply(again, xi)
    torch.cuda.synchronize()
    assert n1 == n2 and n1 > 0 and torch.equal(S1, S2)
    st = sm.stats_get()
    assert st["interp_pairs"] == 2 * 100 * wl.M and st["interp_fallbacks"] == n1 + n2
    model.free()
    again.free()


def test_reduced_basis_model_roundtrip(sm, tmp_path):
    wl = W.MESH8
    xi_tr = torch.from_numpy(W.uniform_xi(64, wl.nxi, 7102)).cuda()
    model = sm.reduce(sm.coef_bumps(xi_tr, wl.nfine, **wl.coef_params()), wl.nc, wl.nc, wl.m)
    path = str(tmp_path / "rb.bin")
    model.save(path)
    again = sm.model_load(path)
    for which in ("r", "lambda", "Z", "phibar"):
        np.testing.assert_array_equal(again.export(which), model.export(which))
    xi = torch.from_numpy(W.uniform_xi(200, wl.nxi, 7103)).cuda()
    a32 = sm.coef_bumps(xi, wl.nfine, **wl.coef_params(), dtype=torch.float32)
    for prec in (sm.PREC_F32, sm.PREC_F64):
        S1 = sm.reduce_apply(model, a32, precision=prec)
        S2 = sm.reduce_apply(again, a32, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(S1, S2)
    model.free()
    again.free()


@pytest.mark.parametrize("base,m,nc", [("mesh8", 8, 8), ("mesh32", 16, 16)])
def test_surrogate_model_roundtrip(sm, tmp_path, base, m, nc):
    import dataclasses

    # m = 8: fused fallback; m = 16: the chunked fallback (bumps of the 32x32
    # family, so that every patch has at most four local variables)
    wl = dataclasses.replace(W.MESH8 if base == "mesh8" else W.MESH32, nc=nc, m=m)
    fam = sm.bump_family(wl)
    lv, _ = sm.local_vars_bumps(wl.nc, wl.nc, wl.m, fam)
    model = sm.mlp_create(wl.nc, wl.nc, wl.m, lv, W.mlp_init(wl.M, 7104), fam, 1.0)
    xi_tr = torch.from_numpy(W.uniform_xi(128, wl.nxi, 7105)).cuda()
    S_tr = sm.upscale(sm.coef_bumps(xi_tr, wl.nfine, **wl.coef_params()), wl.nc, wl.nc, wl.m)
    sm.mlp_set_data(model, xi_tr, S_tr)
    sm.mlp_train(model, 300, 2e-3, torch.from_numpy(W.permutation(128, 7106)).cuda())
    path = str(tmp_path / "mlp.bin")
    model.save(path)
    again = sm.model_load(path)
    torch.cuda.synchronize()
    assert torch.equal(sm.mlp_params(model), sm.mlp_params(again))
    xi = torch.from_numpy(W.uniform_xi(300, wl.nxi, 7107)).cuda()
    st1 = torch.empty((300, wl.M), dtype=torch.int32, device="cuda")
    st2 = torch.empty_like(st1)
    S1 = sm.upscale_surrogate(model, xi, 1e-3, sm.PREC_BF16, status=st1)
    S2 = sm.upscale_surrogate(again, xi, 1e-3, sm.PREC_BF16, status=st2)
    torch.cuda.synchronize()
    assert torch.equal(S1, S2) and torch.equal(st1, st2)
    # a loaded surrogate trains again once it has data
    with pytest.raises(sm.StomsfemError):
        sm.mlp_train(again, 1, 1e-3)
    sm.mlp_set_data(again, xi_tr, S_tr)
    sm.mlp_train(again, 1, 1e-3)
    model.free()
    again.free()


def test_oversampled_reduced_basis_model_roundtrip(sm, tmp_path):
    wl = W.MESH8
    xi_tr = torch.from_numpy(W.uniform_xi(24, wl.nxi, 7104)).cuda()
    model = sm.reduce_os(sm.coef_bumps(xi_tr, wl.nfine, **wl.coef_params()), wl.nc, wl.nc, wl.m, 4)
    path = str(tmp_path / "rb_os.bin")
    model.save(path)
    again = sm.model_load(path)
    assert (again.ncx, again.ncy, again.m) == (wl.nc, wl.nc, wl.m)
    again.patch_m = model.patch_m
    for which in ("r", "lambda", "Z", "phibar"):
        np.testing.assert_array_equal(again.export(which), model.export(which))
    xi = torch.from_numpy(W.uniform_xi(150, wl.nxi, 7105)).cuda()
    a32 = sm.coef_bumps(xi, wl.nfine, **wl.coef_params(), dtype=torch.float32)
    for prec in (sm.PREC_F32, sm.PREC_F64):
        S1 = sm.reduce_os_apply(model, a32, precision=prec)
        S2 = sm.reduce_os_apply(again, a32, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(S1, S2)
    model.free()
    again.free()


def test_model_kinds_are_not_interchangeable(sm):
    # an oversampled reduced-basis model is refused by the other online
    # stages, and the other models by its online stage, before any launch
    wl = W.MESH8
    xi_tr = torch.from_numpy(W.uniform_xi(8, wl.nxi, 7106)).cuda()
    a = sm.coef_bumps(xi_tr, wl.nfine, **wl.coef_params())
    os_model = sm.reduce_os(a, wl.nc, wl.nc, wl.m, 4)
    plain = sm.reduce(a, wl.nc, wl.nc, wl.m)
    S = torch.empty((8, wl.M, 16), dtype=torch.float64, device="cuda")
    kappa = torch.ones((8, wl.nfine, wl.nfine), dtype=torch.float64, device="cuda")
    xi = torch.zeros((8, wl.M, 4), dtype=torch.float64, device="cuda")
    rc = sm.lib().stomsfem_kl_interp_apply(os_model.handle, xi.data_ptr(), kappa.data_ptr(), 8, S.data_ptr(), None,
                                           None, None)
    assert rc == sm.EINVAL
    with pytest.raises(sm.StomsfemError) as e:
        sm.reduce_apply(os_model, a)
    assert e.value.code == sm.EINVAL
    with pytest.raises(sm.StomsfemError) as e:
        sm.reduce_os_apply(plain, a)
    assert e.value.code == sm.EINVAL
    os_model.free()
    plain.free()
