"""Pins of the oracle's oversampling and Petrov-Galerkin path (Sec. 2.2, the
remark on oversampling and eq. stiffness_local_petrov) against facts fixed
outside it: exact reproduction of bilinear fields, the no-oversampling special
case, the zero row and column sums of the local matrices, the nodal
interpolation property of the re-normalised basis, a dense brute-force
construction on tiny patches, LAPACK for the banded LU, and the reduction of
the resonance error against a fine-grid FEM that the remark describes."""
import numpy as np
import pytest

from paper_1607_00693_amd import workloads as W

# textbook Q1 element matrix on a square, CCW nodes (lower left first)
KQ1 = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0


def _field(ncx, ncy, m, seed, lo=0.2, hi=5.0):
    return W.uniform_array((ncy * m, ncx * m), lo, hi, seed)


@pytest.mark.parametrize("m,o", [(4, 2), (8, 4), (8, 8)])
def test_constant_coefficient_gives_the_q1_stiffness(orc, m, o):
    # psi^j are the bilinear functions of the patch, exactly representable, so
    # phi^i are K's bilinear nodal functions and S = a K_Q1 for any patch
    # position (interior, edge, corner, shifted at the domain boundary)
    ncx, ncy = 4, 3
    a = np.full((ncy * m, ncx * m), 2.5)
    for kx, ky in [(0, 0), (1, 1), (3, 2), (2, 0), (0, 2)]:
        S = orc.cell_S_os(a, m, o, kx, ky)
        np.testing.assert_allclose(S, 2.5 * KQ1, rtol=0, atol=1e-13)


def test_no_oversampling_is_the_msfem_stiffness(orc):
    # o = 0: the patch is K, C = I, and the Petrov-Galerkin stiffness equals
    # the Galerkin one (phi^l is a-harmonic, so int a grad phi^l.grad(phi^l' - p^l') = 0)
    m, ncx, ncy = 8, 3, 2
    a = _field(ncx, ncy, m, 11)
    for kx, ky in [(0, 0), (2, 1), (1, 0)]:
        S = orc.cell_S_os(a, m, 0, kx, ky)
        blk = a[ky * m:(ky + 1) * m, kx * m:(kx + 1) * m]
        packed, _ = orc.cell_S(blk)
        np.testing.assert_allclose(S, orc.unpack(packed), rtol=0, atol=1e-12 * np.abs(S).max())


@pytest.mark.parametrize("o", [2, 4])
def test_zero_row_and_column_sums(orc, o):
    # rows: sum_l' p^l' = 1 on K; columns: sum_i phi^i = 1 (the constant is
    # a-harmonic and the normalisation keeps it); both hit a zero gradient
    m, ncx, ncy = 4, 4, 4
    a = _field(ncx, ncy, m, 12 + o, 0.1, 10.0)
    S, st = orc.upscale_os(a[None], ncx, ncy, m, o)
    assert (st == 0).all()
    S = S.reshape(-1, 4, 4)
    sc = np.abs(S).max()
    assert np.abs(S.sum(axis=2)).max() < 1e-12 * sc
    assert np.abs(S.sum(axis=1)).max() < 1e-12 * sc
    # and S is genuinely non-symmetric once the patch is larger than K
    assert np.abs(S - S.transpose(0, 2, 1)).max() > 1e-3 * sc


def test_basis_interpolates_at_the_corners(orc):
    m, o, ncx, ncy = 8, 4, 3, 3
    a = _field(ncx, ncy, m, 21)
    for kx, ky in [(0, 0), (1, 1), (2, 1)]:
        phi, Psi = orc.cell_phi_os(a, m, o, kx, ky)
        corners = [(0, 0), (m, 0), (m, m), (0, m)]  # (px, py), CCW
        for i in range(4):
            for k, (px, py) in enumerate(corners):
                assert abs(phi[i, py, px] - (i == k)) < 1e-12
        np.testing.assert_allclose(phi.sum(axis=0), 1.0, rtol=0, atol=1e-12)
        # the patch solutions are a partition of unity too
        np.testing.assert_allclose(Psi.sum(axis=1), 1.0, rtol=0, atol=1e-12)


def _dense_os_S(a, m, o, kx, ky):
    """Independent brute force: dense patch system, LAPACK solves, explicit inverse."""
    nfy, nfx = a.shape
    mp = m + 2 * o
    x0 = min(max(kx * m - o, 0), nfx - mp)
    y0 = min(max(ky * m - o, 0), nfy - mp)
    ap = a[y0:y0 + mp, x0:x0 + mp]
    nn = mp + 1
    N = nn * nn
    A = np.zeros((N, N))
    for ey in range(mp):
        for ex in range(mp):
            nodes = [ey * nn + ex, ey * nn + ex + 1, (ey + 1) * nn + ex + 1, (ey + 1) * nn + ex]
            A[np.ix_(nodes, nodes)] += ap[ey, ex] * KQ1
    t = np.arange(nn) / mp
    X, Y = np.meshgrid(t, t)
    G = np.stack([(1 - X) * (1 - Y), X * (1 - Y), X * Y, (1 - X) * Y]).reshape(4, N)
    bnd = np.zeros((nn, nn), dtype=bool)
    bnd[0, :] = bnd[-1, :] = bnd[:, 0] = bnd[:, -1] = True
    bnd = bnd.ravel()
    I = ~bnd
    psi = G.copy()
    for j in range(4):
        psi[j, I] = np.linalg.solve(A[np.ix_(I, I)], -A[np.ix_(I, bnd)] @ G[j, bnd])
    cx, cy = kx * m - x0, ky * m - y0
    cn = [cy * nn + cx, cy * nn + cx + m, (cy + m) * nn + cx + m, (cy + m) * nn + cx]
    Psi = psi[:, cn].T  # Psi[k][j]
    Cm = np.linalg.inv(Psi.T)
    kn = np.array([(cy + py) * nn + cx + px for py in range(m + 1) for px in range(m + 1)])
    phi = Cm @ psi[:, kn]  # [4][(m+1)^2] on K
    s = np.arange(m + 1) / m
    XK, YK = np.meshgrid(s, s)
    P = np.stack([(1 - XK) * (1 - YK), XK * (1 - YK), XK * YK, (1 - XK) * YK]).reshape(4, -1)
    S = np.zeros((4, 4))
    mm = m + 1
    for ey in range(m):
        for ex in range(m):
            nodes = [ey * mm + ex, ey * mm + ex + 1, (ey + 1) * mm + ex + 1, (ey + 1) * mm + ex]
            ae = a[ky * m + ey, kx * m + ex]
            S += ae * phi[:, nodes] @ KQ1 @ P[:, nodes].T
    return S


@pytest.mark.parametrize("m,o,ncx,ncy", [(4, 2, 3, 3), (4, 2, 3, 2), (4, 4, 3, 3), (6, 3, 3, 3)])
def test_brute_force_dense(orc, m, o, ncx, ncy):
    a = _field(ncx, ncy, m, 31 + m + o)
    for kx in range(ncx):
        for ky in range(ncy):
            S = orc.cell_S_os(a, m, o, kx, ky)
            ref = _dense_os_S(a, m, o, kx, ky)
            np.testing.assert_allclose(S, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("n,kl,ku,seed", [(30, 4, 4, 1), (57, 8, 8, 2), (12, 3, 5, 3)])
def test_band_lu_against_lapack(orc, n, kl, ku, seed):
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    for i in range(n):
        for c in range(max(0, i - kl), min(n, i + ku + 1)):
            A[i, c] = rng.normal()
    A[np.arange(n), np.arange(n)] *= 0.1  # small pivots: row interchanges happen
    b = rng.normal(size=n)
    x = orc.band_lu_solve(A, b, kl, ku)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-10 * np.abs(x).max())


def test_pg_coarse_solve_symmetric_case(orc):
    # with o = 0 the local matrices are symmetric: the Petrov-Galerkin coarse
    # solve must agree with the symmetric (Cholesky) one
    m, ncx, ncy = 4, 5, 4
    a = _field(ncx, ncy, m, 41)[None]
    S16, _ = orc.upscale_os(a, ncx, ncy, m, 0)
    S10, _, _ = orc.upscale(a, ncx, ncy, m)
    U16, _, _ = orc.coarse_solve_pg(S16, ncx, ncy)
    U10, _, _ = orc.coarse_solve(S10, ncx, ncy)
    np.testing.assert_allclose(U16, U10, rtol=0, atol=1e-12 * np.abs(U10).max())


def test_pg_coarse_solve_dense(orc):
    # the assembled non-symmetric system (row = test node, column = trial
    # node) solved densely
    m, o, ncx, ncy = 4, 2, 4, 3
    a = _field(ncx, ncy, m, 43)
    S16, _ = orc.upscale_os(a[None], ncx, ncy, m, o)
    U, _, _ = orc.coarse_solve_pg(S16, ncx, ncy)
    nix, niy = ncx - 1, ncy - 1
    G = np.zeros((nix * niy, nix * niy))
    b = np.zeros(nix * niy)
    H = 1.0 / ncx
    for ky in range(ncy):
        for kx in range(ncx):
            Sk = S16[0, ky * ncx + kx].reshape(4, 4)
            nodes = [(kx, ky), (kx + 1, ky), (kx + 1, ky + 1), (kx, ky + 1)]
            idx = [(py - 1) * nix + px - 1 if 0 < px < ncx and 0 < py < ncy else -1 for px, py in nodes]
            for te in range(4):
                if idx[te] < 0:
                    continue
                b[idx[te]] += H * H / 4
                for tr in range(4):
                    if idx[tr] >= 0:
                        G[idx[te], idx[tr]] += Sk[tr, te]
    np.testing.assert_allclose(U[0], np.linalg.solve(G, b), rtol=0, atol=1e-12 * np.abs(U).max())


@pytest.mark.parametrize("eps_over_H", [1.0, 1.3])
def test_oversampling_reduces_the_resonance_error(orc, eps_over_H):
    # Sec. 2.2 remark: with the oscillation period close to H the plain MsFEM
    # has a resonance error that oversampling removes.  Reference: the global
    # fine-grid Q1 FEM at the coarse nodes.
    ncx, m = 16, 8
    nf = ncx * m
    x = (np.arange(nf) + 0.5) / nf
    X, Y = np.meshgrid(x, x)
    eps = eps_over_H / ncx
    a = 2.0 + 1.8 * np.sin(2 * np.pi * X / eps) * np.sin(2 * np.pi * Y / eps)
    uf = orc.fine_fem(a).reshape(nf - 1, nf - 1)
    ref = uf[m - 1::m, m - 1::m][:ncx - 1, :ncx - 1]
    err = {}
    for o in (0, m // 2, m):
        S16, _ = orc.upscale_os(a[None], ncx, ncx, m, o)
        U, _, _ = orc.coarse_solve_pg(S16, ncx, ncx)
        err[o] = np.abs(U[0].reshape(ncx - 1, ncx - 1) - ref).max() / np.abs(ref).max()
    assert err[m // 2] < 0.3 * err[0] and err[m] < 0.3 * err[0], err
