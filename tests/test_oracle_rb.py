"""Pins of the reduced-basis oracle (Sec. 3.2) against facts of the method."""
import numpy as np
import pytest

from paper_1607_00693_amd import workloads as W


def _blocks(N, m, seed, sigma=0.8):
    return W.lognormal_field((N, m, m), sigma, seed)


def test_modes_are_energy_orthonormal(orc):
    from oracle import rb
    a = _blocks(40, 6, 1)
    model = rb.rb_offline(a, r_max=10, tail_tol=0.0)
    E, _ = orc.cell_system_dense(model["abar"])
    Z = model["Z"]
    np.testing.assert_allclose(Z.T @ E @ Z, np.eye(Z.shape[1]), atol=1e-10)


def test_full_basis_reproduces_plain(orc):
    # r = n_I: the reduced space is the whole interior space, so the Galerkin
    # solution is the exact cell solution for any coefficient.
    from oracle import rb
    m = 5
    a = _blocks(30, m, 2)
    model = rb.rb_offline(a, r_max=(m - 1) ** 2, tail_tol=0.0)
    assert model["r"] == (m - 1) ** 2
    for s, blk in enumerate(_blocks(3, m, 3, sigma=1.2)):
        S, _ = orc.cell_S(blk)
        np.testing.assert_allclose(rb.rb_online_S(model, blk), S, rtol=0, atol=1e-11 * np.abs(S).max())


def test_training_members_reproduced(orc):
    # three training samples give at most 3*3 - 1 centred snapshot directions;
    # with r >= their rank, every training solution lies in phibar + span(Z)
    # and the Galerkin projection returns it exactly.
    from oracle import rb
    m = 8
    a = _blocks(3, m, 4)
    model = rb.rb_offline(a, r_max=9, tail_tol=1e-13)
    for blk in a:
        S, _ = orc.cell_S(blk)
        np.testing.assert_allclose(rb.rb_online_S(model, blk), S, rtol=0, atol=1e-9 * np.abs(S).max())


def _bump_patch(orc, N, seed, K=(3, 4)):
    # one interior patch of the 8x8-coarse bump workload: four local variables
    wl = W.MESH8
    xi = W.uniform_xi(N, wl.nxi, seed)
    a = orc.coef_bumps(xi, wl.nfine, **wl.coef_params())
    kx, ky = K
    return a[:, ky * 8:(ky + 1) * 8, kx * 8:(kx + 1) * 8].copy()


def test_reduced_energy_dominates_and_decreases(orc):
    # Galerkin on nested subspaces: S_rb(r) - S and S_rb(r) - S_rb(r+2) are
    # PSD; with few local random variables the error falls quickly with r.
    from oracle import rb
    m = 8
    a = _bump_patch(orc, 128, 5)
    test = _bump_patch(orc, 4, 6)
    prev = None
    errs = []
    for r in (2, 4, 6, 8):
        model = rb.rb_offline(a, r_max=r, tail_tol=0.0)
        assert model["r"] == r
        cur = []
        for blk in test:
            S = orc.unpack(orc.cell_S(blk)[0])
            Srb = orc.unpack(rb.rb_online_S(model, blk))
            scale = np.abs(S).max()
            assert np.linalg.eigvalsh(Srb - S).min() > -1e-12 * scale
            cur.append(Srb)
        if prev is not None:
            for p_, c_ in zip(prev, cur):
                assert np.linalg.eigvalsh(p_ - c_).min() > -1e-12 * np.abs(c_).max()
        errs.append(max(np.abs(c_ - orc.unpack(orc.cell_S(b)[0])).max() for c_, b in zip(cur, test)))
        prev = cur
    assert errs[-1] < errs[0] / 100, errs


def test_tail_rule_picks_r(orc):
    from oracle import rb
    a = _blocks(50, 6, 7)
    full = rb.rb_offline(a, r_max=100, tail_tol=0.0)
    sig = full["sigma"]
    tol = 1e-3
    model = rb.rb_offline(a, r_max=100, tail_tol=tol)
    r = model["r"]
    tail = lambda q: np.sqrt(np.sum(sig[q:] ** 2) / np.sum(sig**2))
    assert tail(r) <= tol and tail(r - 1) > tol
    assert rb.rb_offline(a, r_max=3, tail_tol=tol)["r"] == 3
