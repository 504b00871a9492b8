"""Pins of the oracle's two-level Monte Carlo estimator (Sec. 4.1.1, the
remark with eqs. MCmean2level and mseML): the coarse-node gather of the
fine solution against a closed form, the telescoping identity when both
sample sets coincide (M2 = the fine-grid MC mean), the fine FEM against the
m = 1 upscaled system, and unbiasedness against a direct fine-grid Monte
Carlo estimate within the combined standard errors."""
import numpy as np

from oracle import core, twolevel
from paper_1607_00693_amd import workloads as W


def test_gather_picks_the_coinciding_fine_nodes():
    nc, m = 4, 3
    nf = nc * m
    X, Y = np.meshgrid(np.arange(1, nf), np.arange(1, nf))  # fine interior node coordinates
    u = (10 * Y + X).reshape(1, -1).astype(float)
    got = twolevel.fine_at_coarse_nodes(u, nc, m)[0]
    ref = [10 * py * m + px * m for py in range(1, nc) for px in range(1, nc)]
    np.testing.assert_array_equal(got, ref)


def _mesh8_samples(N, seed):
    wl = W.MESH8
    xi = W.uniform_xi(N, wl.nxi, seed)
    a = core.coef_bumps(xi, wl.nfine, **wl.coef_params())
    S, st, _ = core.upscale(a, wl.nc, wl.nc, wl.m)
    U, _, _ = core.coarse_solve(S, wl.nc, wl.nc)
    return a, U


def test_fine_fem_is_the_m1_upscaled_system():
    # the global fine FEM equals the coarse solve of the m = 1 "upscaled"
    # element matrices a_e K_Q1 (independent C routines)
    a = W.uniform_array((2, 16, 16), 0.2, 5.0, 77)
    S, _, _ = core.upscale(a, 16, 16, 1)
    U, _, _ = core.coarse_solve(S, 16, 16)
    for s in range(2):
        np.testing.assert_allclose(core.fine_fem(a[s]), U[s], rtol=0, atol=1e-13 * np.abs(U[s]).max())


def test_same_samples_telescope_to_the_fine_mean():
    wl = W.MESH8
    a, U = _mesh8_samples(12, 501)
    uf = twolevel.fine_solutions(a)
    mean, var_H, var_d, mse = twolevel.two_level(U, U, uf, wl.nc, wl.m)
    np.testing.assert_allclose(mean, twolevel.fine_at_coarse_nodes(uf, wl.nc, wl.m).mean(axis=0), rtol=1e-13)
    assert (var_H >= 0).all() and (var_d >= 0).all() and mse > 0
    # u_H approximates u_h: the correction varies much less than u_H itself
    assert var_d.sum() < 0.05 * var_H.sum()


def test_two_level_is_unbiased_for_the_fine_mean():
    wl = W.MESH8
    _, U_H = _mesh8_samples(8000, 511)
    a2, U_Hh = _mesh8_samples(150, 512)
    M2, var_H, var_d, _ = twolevel.two_level(U_H, U_Hh, twolevel.fine_solutions(a2), wl.nc, wl.m)
    a3, _ = _mesh8_samples(400, 513)
    uh = twolevel.fine_at_coarse_nodes(twolevel.fine_solutions(a3), wl.nc, wl.m)
    se = np.sqrt(var_H / 8000 + var_d / 150 + uh.var(axis=0) / 400)
    assert np.all(np.abs(M2 - uh.mean(axis=0)) < 4.5 * se)
    # and the plain coarse mean is biased by the discretisation error, which
    # the correction term removes: it is larger than the two-level error bar
    bias = np.abs(U_H.mean(axis=0) - M2).max()
    assert bias > 2 * np.sqrt(var_d / 150).max()
