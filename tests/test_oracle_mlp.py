"""Pins of the MLP oracle: finite differences, exact special cases, GELU."""
import math

import numpy as np
import pytest

from paper_1607_00693_amd import workloads as W


def _params(kin, seed, scale=0.5):
    from oracle import mlp
    return W.uniform_array(mlp.nparams(kin), -scale, scale, seed)


def test_gelu_matches_normal_cdf_definition():
    from oracle import mlp
    from scipy.stats import norm
    z = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(mlp.gelu(z), z * norm.cdf(z), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(mlp.gelu_grad(z), norm.cdf(z) + z * norm.pdf(z), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kin", [1, 2, 4])
def test_gradient_matches_central_differences(kin):
    from oracle import mlp
    flat = _params(kin, 10 + kin)
    X = W.uniform_array((7, kin), -1, 1, 20 + kin)
    T = W.uniform_array((7, 10), -2, 2, 30 + kin)
    L, g = mlp.grad(flat, X, T, kin)
    rng = np.random.default_rng(40 + kin)
    idx = rng.choice(flat.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        Lp = mlp.loss(mlp.forward(flat + e, X, kin)[0], T)
        Lm = mlp.loss(mlp.forward(flat - e, X, kin)[0], T)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_zero_weights_give_bias():
    from oracle import mlp
    kin = 4
    ps = mlp.unpack_params(np.zeros(mlp.nparams(kin)), kin)
    ps[-1] = W.uniform_array(20, -1, 1, 3)
    Y, _ = mlp.forward(mlp.pack_params(ps), W.uniform_array((5, kin), -1, 1, 4), kin)
    np.testing.assert_array_equal(Y, np.tile(ps[-1], (5, 1)))


def test_adam_first_step_is_signed_lr():
    # with zero moments, the bias-corrected first Adam step is -lr * sign(g)
    from oracle import mlp
    g = W.uniform_array(50, -3, 3, 5)
    x1, _, _ = mlp.adam_step(np.zeros(50), g, np.zeros(50), np.zeros(50), 1, 0.01, eps=0.0)
    np.testing.assert_allclose(x1, -0.01 * np.sign(g), rtol=1e-12)


def test_gate_accepts_exact_and_rejects_inconsistent(orc):
    from oracle import mlp
    a = W.lognormal_field((3, 8, 8), 0.5, 6)
    S = np.stack([orc.cell_S(b)[0] for b in a])
    mu, sd = S.mean(0), np.maximum(S.std(0), 1e-3)
    Y = np.concatenate([(S - mu) / sd, (S - mu) / sd], axis=1)
    X = np.zeros((3, 4))
    ok, Sp, resid, unc = mlp.gate(Y, mu, sd, X, 4, 1e-3)
    assert ok.all() and resid.max() < 1e-12 and unc.max() == 0
    np.testing.assert_allclose(Sp, S, rtol=0, atol=1e-12 * np.abs(S).max())
    # perturb one head: disagreement; perturb both alike: row-sum residual
    Y2 = Y.copy()
    Y2[0, 10] += 0.1 / sd[0] * np.abs(S[0]).max()
    Y2[1, [0, 10]] += 0.1 / sd[0] * np.abs(S[1]).max()
    X2 = X.copy()
    X2[2, 1] = 1.5
    ok2, _, resid2, unc2 = mlp.gate(Y2, mu, sd, X2, 4, 1e-3)
    assert list(ok2) == [False, False, False]
    assert unc2[0] > 1e-2 and resid2[1] > 1e-2
    assert mlp.gate(Y2, mu, sd, X2, 1, 1e-3)[0][2]   # out-of-box variable not local => accepted


@pytest.mark.parametrize("lr", [0.01, 3e-4])
def test_adam_constant_gradient_moves_lr_per_step(lr):
    # Kingma & Ba: with a constant gradient g, both bias-corrected moment
    # estimates are exact at every step (m_hat = g, v_hat = g^2), so each of
    # the first t steps moves every parameter by -lr * sign(g) (eps = 0).  A
    # slip in either moment update or either bias correction at t >= 2 breaks
    # this.
    from oracle import mlp
    g = W.uniform_array(40, -3, 3, 51)
    x0 = W.uniform_array(40, -1, 1, 52)
    x, m1, m2 = x0.copy(), np.zeros(40), np.zeros(40)
    for t in range(1, 8):
        x, m1, m2 = mlp.adam_step(x, g, m1, m2, t, lr, eps=0.0)
        np.testing.assert_allclose(x, x0 - t * lr * np.sign(g), rtol=0, atol=1e-12)


def test_adam_is_invariant_to_gradient_scale():
    # the update depends on m_hat / sqrt(v_hat): scaling every gradient by
    # c > 0 leaves the whole trajectory unchanged (eps = 0)
    from oracle import mlp
    gs = [W.uniform_array(30, -2, 2, 60 + t) for t in range(6)]
    for c in (1e-3, 7.0):
        xa, xb = np.zeros(30), np.zeros(30)
        ma = [np.zeros(30), np.zeros(30)]
        mb = [np.zeros(30), np.zeros(30)]
        for t, g in enumerate(gs, start=1):
            xa, ma[0], ma[1] = mlp.adam_step(xa, g, ma[0], ma[1], t, 1e-2, eps=0.0)
            xb, mb[0], mb[1] = mlp.adam_step(xb, c * g, mb[0], mb[1], t, 1e-2, eps=0.0)
            np.testing.assert_allclose(xb, xa, rtol=1e-12, atol=1e-15)


def test_standardize_recovers_affine_targets_and_floors_constants():
    # targets alpha_q + beta_q * u with u of mean 0 and population standard
    # deviation 1 (u = +-1 alternating): mean alpha, std |beta| (1/N form,
    # not 1/(N-1)); a constant entry gets the floor 1e-12 max(1, max|mean|)
    from oracle import mlp
    N = 50
    u = np.where(np.arange(N) % 2 == 0, 1.0, -1.0)
    alpha = W.uniform_array(10, -5, 5, 70)
    beta = W.uniform_array(10, -2, 2, 71)
    beta[3] = 0.0
    S = alpha[None, :] + beta[None, :] * u[:, None]
    mu, sd = mlp.standardize(S)
    np.testing.assert_allclose(mu, alpha, rtol=0, atol=1e-14)
    expect = np.abs(beta)
    expect[3] = 1e-12 * max(1.0, np.abs(alpha).max())
    np.testing.assert_allclose(sd, expect, rtol=1e-14, atol=0)


def test_gate_rejects_non_finite_predictions():
    # a NaN or an infinite de-standardised value must never be accepted
    from oracle import mlp
    mu = np.linspace(1.0, 2.0, 10)
    sd = np.full(10, 0.1)
    Y = np.zeros((4, 20))
    Y[1, 3] = np.nan
    Y[2, 15] = np.inf
    Y[3, 0] = -np.inf
    ok, _, resid, unc = mlp.gate(Y, mu, sd, np.zeros((4, 4)), 4, 1e30)
    assert ok.tolist() == [True, False, False, False]
    assert np.isnan(resid[1:]).all() and np.isnan(unc[1:]).all()


def test_gate_output_scale_is_a_pure_rescaling(orc):
    # the network predicts S / c: the gate multiplies both heads by c, so the
    # accepted S is the exact one and the two signals do not depend on c
    from oracle import mlp
    a = W.lognormal_field((4, 8, 8), 1.0, 16)
    S = np.stack([orc.cell_S(b)[0] for b in a])
    c = np.array([1.0, 3.5, 250.0, 1e4])
    mu, sd = (S / c[:, None]).mean(0), np.maximum((S / c[:, None]).std(0), 1e-3)
    T = (S / c[:, None] - mu) / sd
    ok, Sp, resid, unc = mlp.gate(np.concatenate([T, T], 1), mu, sd, np.zeros((4, 4)), 4, 1e-3, scale=c)
    assert ok.all()
    np.testing.assert_allclose(Sp, S, rtol=0, atol=1e-12 * np.abs(S).max())
    Y = np.concatenate([T, T + W.uniform_array(T.shape, -1e-3, 1e-3, 17)], 1)
    r1 = mlp.gate(Y, mu, sd, np.zeros((4, 4)), 4, 1e-3, scale=c)
    r0 = mlp.gate(Y, mu, sd, np.zeros((4, 4)), 4, 1e-3)
    np.testing.assert_allclose(r1[2], r0[2], rtol=1e-13)
    np.testing.assert_allclose(r1[3], r0[3], rtol=1e-13)
    np.testing.assert_allclose(r1[1], c[:, None] * r0[1], rtol=1e-13, atol=0)


def test_ring_mean_hand_counted():
    from oracle import mlp
    blk = np.ones((3, 3))
    blk[1, 1] = 100.0                       # the only interior element
    assert mlp.ring_mean(blk) == 1.0
    assert mlp.ring_mean(np.array([[7.0]])) == 7.0
    m, th = 8, 1234.5
    blk = np.ones((m, m))
    blk[3, :] = th                          # a channel across the patch: 2 of 4m-4 ring elements
    assert abs(mlp.ring_mean(blk) - (1 + 2 * (th - 1) / (4 * m - 4))) < 1e-12 * th
    blk = np.ones((m, m))
    blk[0, :] = th                          # along an edge: m of 4m-4
    assert abs(mlp.ring_mean(blk) - (1 + m * (th - 1) / (4 * m - 4))) < 1e-12 * th


def test_features_input_recovers_the_conductivity(orc):
    # theta = 10^(d (u + 1) / 2) with u the network input of the variable,
    # against the oracle's coefficient of a single square inclusion
    from oracle import mlp
    xs = np.array([[-3.0], [-0.4], [0.0], [1.7], [3.0]])
    a = orc.coef_features(xs, 8, [2], [0.5], [0.5], [0.2], decades=4.0)
    th = a[:, 4, 4]
    u = mlp.features_input(xs[:, 0])
    np.testing.assert_allclose(10.0 ** (4.0 * (u + 1.0) / 2.0), th, rtol=1e-13)
    assert (np.abs(u) < 1).all() and u[2] == 0.0


def test_ring_mean_follows_max_entry_of_S_across_decades(orc):
    # the premise of the output scale: for a channel across the patch, an
    # edge channel and an interior inclusion, max|S| / ring mean stays within
    # a factor 3 while the conductivity runs over four decades
    from oracle import mlp
    m = 8
    shapes = []
    b = np.zeros((m, m), bool); b[3, :] = True; shapes.append(b)
    b = np.zeros((m, m), bool); b[0, 2:] = True; shapes.append(b)
    b = np.zeros((m, m), bool); b[2:6, 2:6] = True; shapes.append(b)
    spread = []
    for mask in shapes:
        ratios, mx = [], []
        for th in 10.0 ** np.linspace(0.2, 3.8, 7):
            blk = np.where(mask, th, 1.0)
            S, _ = orc.cell_S(blk)
            mx.append(np.abs(S).max())
            ratios.append(mx[-1] / mlp.ring_mean(blk))
        assert max(ratios) / min(ratios) < 3.0
        spread.append(max(mx) / min(mx))
    assert spread[0] > 50 and spread[1] > 50 and spread[2] < 10   # channels grow, the inclusion saturates
