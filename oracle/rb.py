"""Reduced-basis oracle (Sec. 3.2: eqs. KLphi, localRB, localRBsystem;
Algorithms 3 and 4).  Test infrastructure only (see package doc).

Offline, per coarse element (patch):
  1. cell-problem solutions phi^l(xi_s), l = 0, 1, 2, at the training samples;
  2. their mean phibar^l;
  3. centred snapshots Psi = [phi^l(xi_s) - phibar^l] (interior nodes, the
     three l stacked side by side, one shared basis per patch);
  4. the energy inner product of H^1_0(K; abar), abar = training mean of the
     coefficient: E = K_II(abar);
  5. E = R^T R (Cholesky), SVD of R Psi (the KL expansion in that inner
     product);
  6. r = min(r_max, smallest r whose relative tail
     sqrt(sum_{q>r} s_q^2 / sum_q s_q^2) <= tail_tol, number of s_q^2 above
     RANK_TOL s_0^2: the numerical rank of the snapshots);
  7. modes Z = R^{-1} U_r, so that Z^T E Z = I.
Online, per (patch, sample): the Galerkin system of eq. localRBsystem,
  A = Z^T K_II(a) Z,  F^l = -Z^T (K_II(a) phibar^l + K_IB(a) g^l),
  c^l = A^{-1} F^l,   phi_rb^l = phibar^l + Z c^l  (boundary data g^l),
  phi_rb^3 = 1 - sum_l phi_rb^l,
and S_rb by the element sum of eq. stiffness_local.

numpy's Cholesky, SVD and solve are the library steps; the local matrices and
snapshots come from the C oracle.
"""
from __future__ import annotations

import numpy as np

from . import core

RANK_TOL = 1e-12


def _interior(phi_full: np.ndarray) -> np.ndarray:
    """[.., m+1, m+1] nodal field -> interior values [.., (m-1)^2] (natural order)."""
    return phi_full[..., 1:-1, 1:-1].reshape(phi_full.shape[:-2] + (-1,))


def boundary_data(m: int, a_blk: np.ndarray, bc: int) -> np.ndarray:
    """Nodal fields [4][m+1][m+1] that carry the cell-problem Dirichlet data on
    the boundary (their interior values are irrelevant here)."""
    if bc == core.BC_LINEAR:
        t = np.arange(m + 1) / m
        X, Y = np.meshgrid(t, t)
        return np.stack([(1 - X) * (1 - Y), X * (1 - Y), X * Y, (1 - X) * Y])
    return core.cell_phi(a_blk, bc)


def rb_offline(a_train: np.ndarray, r_max: int = 8, tail_tol: float = 1e-6, bc: int = core.BC_LINEAR) -> dict:
    """a_train: [N_train][m][m] coefficient blocks of one patch."""
    Ntr, m, _ = a_train.shape
    nI = (m - 1) ** 2
    phis = np.stack([core.cell_phi(a_train[s], bc) for s in range(Ntr)])  # [N][4][m+1][m+1]
    phi_I = _interior(phis[:, :3])                                        # [N][3][nI]
    phibar = phi_I.mean(axis=0)                                           # [3][nI]
    Psi = (phi_I - phibar[None]).transpose(2, 1, 0).reshape(nI, 3 * Ntr)  # columns (l, s)
    abar = a_train.mean(axis=0)
    E, _ = core.cell_system_dense(abar, bc)
    R = np.linalg.cholesky(E).T                                           # E = R^T R
    U, sig, _ = np.linalg.svd(R @ Psi, full_matrices=False)
    tot = np.sum(sig**2)
    r = None
    for q in range(1, len(sig) + 1):
        tail = np.sqrt(np.sum(sig[q:] ** 2) / tot) if tot > 0 else 0.0
        if tail <= tail_tol:
            r = q
            break
    if r is None:
        r = len(sig)
    r = min(r, r_max, len(sig))
    # numerical rank: modes whose eigenvalue sigma^2 is at or below 1e-12 of
    # the largest are rounding, not part of the snapshot space
    rank = int(np.sum(sig**2 > RANK_TOL * sig[0] ** 2)) if len(sig) and sig[0] > 0 else 0
    r = min(r, rank)
    Z = np.linalg.solve(R, U[:, :r])                                      # R^{-1} U_r
    return {"m": m, "r": r, "Z": Z, "phibar": phibar, "abar": abar, "sigma": sig, "bc": bc}


def rb_online_phi(model: dict, a_blk: np.ndarray) -> np.ndarray:
    """Reduced-basis cell solutions on the full (m+1)^2 grid: [4][m+1][m+1]."""
    m, Z, phibar, bc = model["m"], model["Z"], model["phibar"], model["bc"]
    K, lift = core.cell_system_dense(a_blk, bc)       # lift^l = -K_IB g^l
    A = Z.T @ K @ Z
    phi = np.zeros((4, m + 1, m + 1))
    g = boundary_data(m, a_blk, bc)
    for l in range(3):
        F = Z.T @ (lift[l] - K @ phibar[l])
        c = np.linalg.solve(A, F)
        inner = phibar[l] + Z @ c
        phi[l] = g[l]
        phi[l, 1:-1, 1:-1] = inner.reshape(m - 1, m - 1)
    phi[3] = 1.0 - phi[0] - phi[1] - phi[2]
    return phi


def rb_online_S(model: dict, a_blk: np.ndarray) -> np.ndarray:
    """Packed S_rb[10] by the element sum of eq. stiffness_local."""
    phi = rb_online_phi(model, a_blk)
    return core.pack(core.energy_S(a_blk, phi))


# --- reduced basis on oversampled patches (Secs. 2.2 and 3.2 together; the
# high-contrast example of Sec. 5.2 combines them with the Petrov-Galerkin
# stiffness) -----------------------------------------------------------------
# The cell problems of element K are posed on its oversampled patch (side
# M = m + 2o, moved inside the domain at the edge, core.os_origin) with the
# bilinear data of the patch corners; the reduced basis of the patch is built
# from those patch solutions exactly as above (rb_offline on the patch
# blocks).  Online, the reduced patch solutions psi^j (j = 0..3, psi^3 = 1 -
# sum) give, as in the plain oversampled stiffness: Psi[k][j] = psi^j at the
# corners x_k of K (CCW from the lower left), C = Psi^{-T}, the multiscale
# trial functions phi^i = sum_j C[i][j] psi^j on K, and
#   S16[l][l'] = int_K a grad phi^l . grad p^l'   (p^l': K's bilinear functions)
# by the element sum over K.


def patch_block(a: np.ndarray, K: int, ncx: int, ncy: int, m: int, o: int) -> np.ndarray:
    """The oversampled patch [M][M] of element K of one sample's field a."""
    nfx, nfy = ncx * m, ncy * m
    kx, ky = K % ncx, K // ncx
    x0, y0 = core.os_origin(kx, m, o, nfx), core.os_origin(ky, m, o, nfy)
    M = m + 2 * o
    return a[y0:y0 + M, x0:x0 + M]


def rb_os_online_S16(model: dict, a_patch: np.ndarray, m: int, cx: int, cy: int) -> np.ndarray:
    """S16 [4][4] (row: trial l, column: bilinear test l') of the element whose
    lower-left node is patch node (cx, cy), from the reduced patch solutions."""
    psi = rb_online_phi(model, a_patch)                     # [4][M+1][M+1]
    kx = [cx, cx + m, cx + m, cx]
    ky = [cy, cy, cy + m, cy + m]
    Psi = np.array([[psi[j, ky[k], kx[k]] for j in range(4)] for k in range(4)])
    C = np.linalg.inv(Psi.T)
    phiK = np.einsum("ij,jyx->iyx", C, psi[:, cy:cy + m + 1, cx:cx + m + 1])
    t = np.arange(m + 1) / m
    X, Y = np.meshgrid(t, t)
    test = np.stack([(1 - X) * (1 - Y), X * (1 - Y), X * Y, (1 - X) * Y])
    return core.energy_S(np.ascontiguousarray(a_patch[cy:cy + m, cx:cx + m]), phiK, test)


def rb_os(a_train: np.ndarray, a: np.ndarray, ncx: int, ncy: int, m: int, o: int, r_max: int = 8,
          tail_tol: float = 1e-6):
    """Per element: offline on the training fields' patches, online S16 for
    every sample of a.  Returns (S16 [N][ncy*ncx][16], r [ncy*ncx])."""
    N = a.shape[0]
    Mc = ncx * ncy
    S = np.zeros((N, Mc, 16))
    rs = np.zeros(Mc, dtype=np.int64)
    for K in range(Mc):
        blocks = np.stack([patch_block(a_train[s], K, ncx, ncy, m, o) for s in range(a_train.shape[0])])
        model = rb_offline(np.ascontiguousarray(blocks), r_max, tail_tol)
        rs[K] = model["r"]
        kx, ky = K % ncx, K // ncx
        cx = kx * m - core.os_origin(kx, m, o, ncx * m)
        cy = ky * m - core.os_origin(ky, m, o, ncy * m)
        for s in range(N):
            S[s, K] = rb_os_online_S16(model, np.ascontiguousarray(patch_block(a[s], K, ncx, ncy, m, o)), m, cx,
                                       cy).ravel()
    return S, rs
