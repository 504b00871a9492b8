"""Random-interpolation oracle (Sec. 3.1, Algorithms 1 and 2; accuracy in
Sec. 3.1.1, Thm. 3.3).  Test infrastructure only (see package doc).

Offline, per patch K with local variables xi_K = (xi_{j_0}, ..., xi_{j_{k-1}})
(the bumps whose support holds a fine-element centroid of K, increasing j):
  1. the 1-D node set: nn = nu + 1 Chebyshev-Gauss-Lobatto points
     t_j = cos(pi j / nu), j = 0..nu, mapped affinely from [-1, 1] to the box
     [lo, hi] of the variables;
  2. the tensor grid of the k variables, nn^k nodes, node index
     c = sum_i d_i nn^(k-1-i) (variable 0 varies slowest);
  3. S_K at every node by the plain cell solves (the variables that are not
     local to K do not change the coefficient on K; they are set to 0);
  4. the interpolant of every one of the 10 entries is the tensor Lagrange
     polynomial through those values.
Online, per (sample, patch): read the local variables, evaluate
  S_K(x) = sum_c prod_i l_{d_i}(x_i) S_K(node c),
  l_d(x) = prod_{e != d} (x - t_e) / (t_d - t_e)   (Lagrange basis),
or, when a local variable lies outside [lo, hi], compute S_K directly by the
plain path (the remark after Algorithm 2 of Sec. 3.1).

The load b_K does not depend on xi here (Petrov-Galerkin load, f = 1), so only
S is interpolated.  The plain S and the coefficient come from the C oracle.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import core


def cgl_nodes(nn: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """The nn Chebyshev-Gauss-Lobatto points of [lo, hi], t_0 = hi > ... > t_nu = lo."""
    if nn < 2:
        raise ValueError("need at least two nodes per variable")
    t = np.cos(np.pi * np.arange(nn) / (nn - 1))
    return lo + (t + 1.0) * (hi - lo) / 2.0


def lagrange_basis(x: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """l_d(x) for every d: [len(x)][nn], straight from the product formula."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nn = len(nodes)
    B = np.ones((len(x), nn))
    for d in range(nn):
        for e in range(nn):
            if e != d:
                B[:, d] *= (x - nodes[e]) / (nodes[d] - nodes[e])
    return B


def local_vars_bumps(nc: int, m: int, g: int, rho: float) -> list[list[int]]:
    """Local variables of every patch of the nc x nc mesh (Sec. 3, eq. MsFEB2):
    j is local to K iff some fine-element centroid of K lies strictly inside
    bump j's support disc.  K = ky*nc + kx, j = jy*g + jx."""
    nf = nc * m
    out = []
    for K in range(nc * nc):
        kx, ky = K % nc, K // nc
        c = (np.arange(m) + 0.5) / nf
        xs, ys = np.meshgrid(kx * m / nf + c, ky * m / nf + c)
        js = []
        for j in range(g * g):
            cx, cy = (j % g + 0.5) / g, (j // g + 0.5) / g
            if np.any(((xs - cx) ** 2 + (ys - cy) ** 2) / rho**2 < 1.0):
                js.append(j)
        out.append(js)
    return out


def node_xi(nxi: int, lv: list[int], digits, nodes: np.ndarray) -> np.ndarray:
    """The full random vector of one tensor node of a patch: local variable
    lv[i] takes nodes[digits[i]], every other variable is 0."""
    xi = np.zeros(nxi)
    for i, j in enumerate(lv):
        xi[j] = nodes[digits[i]]
    return xi


def patch_S(xi: np.ndarray, K: int, nc: int, m: int, fam: dict) -> np.ndarray:
    """Plain S_K [N][10] for the full random vectors xi [N][nxi] (the whole
    coefficient field is generated; only patch K's block is upscaled)."""
    xi = np.atleast_2d(xi)
    a = core.coef_bumps(xi, nc * m, fam["g"], fam["rho"], fam["eps"], fam["base"], fam["amp"], fam["beta"])
    kx, ky = K % nc, K // nc
    blk = np.ascontiguousarray(a[:, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m])
    S, st, _ = core.upscale(blk, 1, 1, m)
    if np.any(st != 0):
        raise RuntimeError("plain solve failed at an interpolation node")
    return S[:, 0, :]


def ri_offline(nc: int, m: int, fam: dict, local_vars: list[list[int]], nn: int, lo: float, hi: float,
               patches=None) -> dict:
    """Tables T[K] = S_K at the nn^k tensor nodes, [nn^k][10] (Algorithm 1)."""
    nodes = cgl_nodes(nn, lo, hi)
    nxi = fam["g"] ** 2
    tables = {}
    for K in (range(nc * nc) if patches is None else patches):
        lv = local_vars[K]
        xs = np.array([node_xi(nxi, lv, d, nodes) for d in itertools.product(range(nn), repeat=len(lv))])
        tables[K] = patch_S(xs, K, nc, m, fam)
    return dict(nodes=nodes, nn=nn, lo=lo, hi=hi, tables=tables, local_vars=local_vars)


def ri_eval(table: np.ndarray, nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Tensor Lagrange interpolant of every entry at the points x [N][k]:
    sum over nodes of the product of the 1-D basis values, [N][10]."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, k = x.shape
    nn = len(nodes)
    T = table.reshape((nn,) * k + (table.shape[-1],))
    bases = [lagrange_basis(x[:, i], nodes) for i in range(k)]
    out = np.zeros((N, table.shape[-1]))
    for d in itertools.product(range(nn), repeat=k):
        w = np.ones(N)
        for i in range(k):
            w = w * bases[i][:, d[i]]
        out += w[:, None] * T[d][None, :]
    return out


def ri_online(model: dict, xi: np.ndarray, nc: int, m: int, fam: dict):
    """Algorithm 2 for every sample and patch: (S [N][M][10], fallback mask
    [N][M]); pairs with a local variable outside the box are solved plainly."""
    xi = np.atleast_2d(xi)
    N = xi.shape[0]
    M = nc * nc
    S = np.zeros((N, M, 10))
    fb = np.zeros((N, M), dtype=bool)
    lo, hi = model["lo"], model["hi"]
    for K in range(M):
        lv = model["local_vars"][K]
        x = xi[:, lv]
        inside = np.all((x >= lo) & (x <= hi), axis=1)
        if np.any(inside):
            S[inside, K] = ri_eval(model["tables"][K], model["nodes"], x[inside])
        if np.any(~inside):
            S[~inside, K] = patch_S(xi[~inside], K, nc, m, fam)
            fb[~inside, K] = True
    return S, fb
