"""Two-level Monte Carlo estimator (Sec. 4.1.1, the remark after
eq. umeanMSE: eqs. MCmean2level and mseML).  Test infrastructure only (see
package doc).

  M2[u] = (1/N_H) sum_i u_H(omega_{i,H}) + (1/N_h) sum_i [u_h - u_H](omega_{i,h})

with independent sample sets; u_H is the coarse (StoMsFEM) solution and u_h
the fine-grid FEM solution.  Both are compared at the interior coarse nodes:
u_H there is the coarse nodal value (the multiscale basis is nodal), u_h the
value at the fine node that coincides with the coarse node (fine node
(px m, py m) of coarse node (px, py)).  The sampling part of the MSE is
estimated from the two sample variances, with int_D g ~ H^2 sum over the
interior coarse nodes:

  H^2 sum_nodes ( var[u_H] / N_H + var[u_H - u_h] / N_h ).

Variances use the 1/N normalisation of the Monte Carlo estimator
(M[u^2] - M[u]^2).  The fine solution itself comes from the C oracle's
global Q1 FEM (core.fine_fem).
"""
from __future__ import annotations

import numpy as np

from . import core


def fine_at_coarse_nodes(u_fine: np.ndarray, nc: int, m: int) -> np.ndarray:
    """[N][(nc-1)^2] values of fine interior solutions [N][(nc m - 1)^2] at
    the interior coarse nodes, natural order (x fastest)."""
    u_fine = np.atleast_2d(u_fine)
    nf1 = nc * m - 1
    idx = [(py * m - 1) * nf1 + (px * m - 1) for py in range(1, nc) for px in range(1, nc)]
    return u_fine[:, idx]


def fine_solutions(a: np.ndarray) -> np.ndarray:
    """Fine-grid FEM solutions for coefficient samples a [N][nf][nf]."""
    return np.stack([core.fine_fem(a[s]) for s in range(a.shape[0])])


def two_level(U_H: np.ndarray, U_Hh: np.ndarray, u_fine: np.ndarray, nc: int, m: int):
    """(M2 [nU], var[u_H] [nU], var[u_H - u_h] [nU], sampling MSE estimate)
    from coarse solutions U_H [N_H][nU] of the first sample set, coarse
    solutions U_Hh [N_h][nU] and fine solutions u_fine [N_h][(nc m-1)^2] of
    the second."""
    uh = fine_at_coarse_nodes(u_fine, nc, m)
    d = uh - U_Hh
    mean = U_H.mean(axis=0) + d.mean(axis=0)
    var_H = (U_H * U_H).mean(axis=0) - U_H.mean(axis=0) ** 2
    var_d = (d * d).mean(axis=0) - d.mean(axis=0) ** 2
    H = 1.0 / nc
    mse = H * H * float(np.sum(var_H / U_H.shape[0] + var_d / U_Hh.shape[0]))
    return mean, var_H, var_d, mse
