"""Pins of the reduced basis on oversampled patches (oracle): the reduced
Petrov-Galerkin stiffness of a training sample, whose patch solutions lie in
the reduced space when no mode is truncated, equals the oversampled solve of
that sample (core.upscale_os); with all modes (3 (N_train - 1) >= interior
unknowns) it equals it for any sample; without oversampling and with all modes
it is the plain element stiffness of the C oracle; rows and columns sum to
zero at any rank; on a medium with few local variables the error falls by
orders of magnitude with the rank."""
import numpy as np

from oracle import core, rb
from paper_1607_00693_amd import workloads as W


def _rel(A, B):
    return np.abs(A - B).max() / np.abs(B).max()


def test_training_samples_are_reproduced():
    m, o, nc, N = 4, 2, 3, 4
    a_tr = W.uniform_array((N, nc * m, nc * m), 0.3, 4.0, 3101)
    S_rb, rs = rb.rb_os(a_tr, a_tr, nc, nc, m, o, r_max=3 * N, tail_tol=0.0)
    S_os, _ = core.upscale_os(a_tr, nc, nc, m, o)
    assert _rel(S_rb, S_os) < 1e-10


def test_full_rank_basis_matches_the_oversampled_solve():
    # patch of 8 cells: 49 interior unknowns; the centred snapshots of 18
    # training samples span 3 * 17 = 51 >= 49 directions
    m, o, nc = 4, 2, 3
    a_tr = W.uniform_array((18, nc * m, nc * m), 0.3, 4.0, 3102)
    a = W.uniform_array((2, nc * m, nc * m), 0.3, 4.0, 3103)
    S_rb, rs = rb.rb_os(a_tr, a, nc, nc, m, o, r_max=49, tail_tol=0.0)
    assert (rs == 49).all()
    S_os, _ = core.upscale_os(a, nc, nc, m, o)
    assert _rel(S_rb, S_os) < 1e-9


def test_no_oversampling_full_rank_is_the_plain_cell_solve():
    # o = 0: the patch is the element, Psi = I, and with every interior mode
    # kept the reduced solution is the exact one, whose Petrov-Galerkin and
    # Galerkin energies agree: S16 = the plain element stiffness (C oracle)
    m, nc = 4, 2
    a_tr = W.uniform_array((4, nc * m, nc * m), 0.3, 4.0, 3104)
    a = W.uniform_array((2, nc * m, nc * m), 0.3, 4.0, 3105)
    S_rb, rs = rb.rb_os(a_tr, a, nc, nc, m, 0, r_max=9, tail_tol=0.0)
    assert (rs == 9).all()
    S_pl, _, _ = core.upscale(a, nc, nc, m)
    for s in range(2):
        for K in range(nc * nc):
            assert _rel(S_rb[s, K].reshape(4, 4), core.unpack(S_pl[s, K])) < 1e-10


def test_rows_and_columns_sum_to_zero_at_any_rank():
    # the trial functions and the bilinear test functions each sum to one on
    # the element, for any reduced space: every row and column of S16 sums to 0
    m, o, nc = 4, 2, 3
    a_tr = W.uniform_array((6, nc * m, nc * m), 0.3, 4.0, 3108)
    a = W.uniform_array((2, nc * m, nc * m), 0.3, 4.0, 3109)
    for r in (1, 3, 7):
        S_rb, _ = rb.rb_os(a_tr, a, nc, nc, m, o, r_max=r, tail_tol=0.0)
        S4 = S_rb.reshape(2, nc * nc, 4, 4)
        scale = np.abs(S4).max()
        assert np.abs(S4.sum(-1)).max() < 1e-12 * scale
        assert np.abs(S4.sum(-2)).max() < 1e-12 * scale


def test_error_falls_with_the_rank_on_few_local_variables():
    # bump medium of the 8x8 mesh (16 variables over the domain, a patch of
    # side 2H sees a few of them): the reduced stiffness converges to the
    # oversampled solve as modes are added
    wl = W.MESH8
    m, o, nc = 8, 4, 8
    a_tr = core.coef_bumps(W.uniform_xi(64, wl.nxi, 3201), wl.nfine, **wl.coef_params())
    a = core.coef_bumps(W.uniform_xi(2, wl.nxi, 3202), wl.nfine, **wl.coef_params())
    S_os, _ = core.upscale_os(a, nc, nc, m, o)
    e2 = _rel(rb.rb_os(a_tr, a, nc, nc, m, o, r_max=2, tail_tol=0.0)[0], S_os)
    e32 = _rel(rb.rb_os(a_tr, a, nc, nc, m, o, r_max=32, tail_tol=0.0)[0], S_os)
    assert e32 < e2 / 100, (e2, e32)


def test_degenerate_training_sets_keep_the_numerical_rank():
    # one sample: the centred snapshots vanish, r = 0 and psi = phibar, which
    # is that sample's own patch solution; two samples: the centred snapshots
    # of the two are opposite, rank 3 -- both reproduce their training
    # samples exactly
    m, o, nc = 4, 2, 3
    for N, r_expect in ((1, 0), (2, 3)):
        a = W.uniform_array((N, nc * m, nc * m), 0.3, 4.0, 3110 + N)
        S_rb, rs = rb.rb_os(a, a, nc, nc, m, o, r_max=8, tail_tol=0.0)
        assert (rs == r_expect).all()
        S_os, _ = core.upscale_os(a, nc, nc, m, o)
        assert _rel(S_rb, S_os) < 1e-12
