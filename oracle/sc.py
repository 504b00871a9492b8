"""Global sparse-grid stochastic collocation with search-and-plug-in
dictionaries (Sec. 4.1.2, global SC methods: eqs. sparseintegration,
SCofflinecost, SConlinecost; Sec. 5.2).  Test
infrastructure only (see package doc).

Quadrature.  The random variables are independent and uniform on the box
[lo, hi] (the bump family: U[-1, 1]), so E[f] is the integral of f against
the uniform probability density.  The one-dimensional rules are the nested
Clenshaw-Curtis rules: level 1 is the midpoint with weight 1, level i >= 2
has n_i = 2^(i-1) + 1 points t_j = cos(pi j / (n_i - 1)) (mapped affinely to
the box) and the interpolatory weights, w_j = the mean over the box of the
Lagrange basis polynomial l_j.  The sparse grid of level L in d variables is
Smolyak's combination of tensor products of these rules,

    A(L, d) = sum over multi-indices i (i_k >= 1) with
              max(d, L + 1) <= |i| <= L + d  of
              (-1)^(L + d - |i|) binom(d - 1, L + d - |i|) Q_i1 x ... x Q_id,

and because the rules are nested the union of the tensor grids is the point
set; the weight of a point is the sum of its weights in the terms.

Points are stored as integer digits on the finest one-dimensional grid of
the level, D = 2^max(L, 1) intervals: digit c stands for cos(pi c / D).  A
point of the level-i rule with index j has digit j D / (n_i - 1) (the level-1
midpoint: D / 2).  Node values: x = lo + (cos(pi c / D) + 1)(hi - lo) / 2.
Point sets are sorted lexicographically by digits.

Dictionaries.  The coefficient on a patch K depends only on K's local
variables, so the upscaled S_K at a global collocation point depends only on
the point's digits at those variables: the local collocation point.  Offline,
S_K is computed once per distinct local point (with every non-local variable
set to 0); online, every global point looks its local points up (search) and
takes the stored S_K (plug-in), then assembles and solves the coarse system.
The estimates are E[u_H] ~ sum_p w_p u_H(p) and
var[u_H] ~ sum_p w_p u_H(p)^2 - (sum_p w_p u_H(p))^2.
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np

from . import core
from . import ri


def cc_npoints(i: int) -> int:
    """Number of points of the level-i nested Clenshaw-Curtis rule (i >= 1)."""
    return 1 if i == 1 else 2 ** (i - 1) + 1


def cc_rule(i: int) -> tuple[np.ndarray, np.ndarray]:
    """Points t_j = cos(pi j / (n - 1)) on [-1, 1] and interpolatory weights
    for the uniform probability measure: w_j = (1/2) int_{-1}^{1} l_j(t) dt,
    each l_j integrated exactly by a Gauss-Legendre rule of enough points."""
    n = cc_npoints(i)
    if n == 1:
        return np.zeros(1), np.ones(1)
    t = np.cos(np.pi * np.arange(n) / (n - 1))
    gx, gw = np.polynomial.legendre.leggauss(n)  # exact to degree 2n - 1 >= n - 1
    L = ri.lagrange_basis(gx, t)  # [len(gx)][n]
    return t, 0.5 * (gw @ L)


def digit_base(level: int) -> int:
    """D = 2^max(level, 1): intervals of the finest one-dimensional grid."""
    return 2 ** max(level, 1)


def smolyak_terms(d: int, level: int):
    """(coefficient, multi-index) of every term of the combination formula."""
    q = level + d
    for extra in range(max(0, level - d + 1), level + 1):  # |i| - d
        c = (-1) ** (level - extra) * comb(d - 1, level - extra)
        # multi-indices i >= 1 with |i| = d + extra
        for cut in itertools.combinations(range(extra + d - 1), d - 1):
            parts = []
            prev = -1
            for b in cut + (extra + d - 1,):
                parts.append(b - prev - 1)
                prev = b
            yield c, tuple(p + 1 for p in parts)
    assert q == level + d


def sparse_grid(d: int, level: int) -> tuple[np.ndarray, np.ndarray]:
    """Digits [n][d] (int, sorted lexicographically) and weights [n] of the
    level-`level` Smolyak Clenshaw-Curtis grid for the uniform probability
    measure on the d-dimensional box."""
    if d < 1 or level < 0:
        raise ValueError("need d >= 1 and level >= 0")
    D = digit_base(level)
    acc: dict[tuple, float] = {}
    for c, idx in smolyak_terms(d, level):
        rules = []
        for i in idx:
            n = cc_npoints(i)
            _, w = cc_rule(i)
            digs = [D // 2] if n == 1 else [j * D // (n - 1) for j in range(n)]
            rules.append(list(zip(digs, w)))
        for combo in itertools.product(*rules):
            key = tuple(dg for dg, _ in combo)
            wt = c * float(np.prod([w for _, w in combo]))
            acc[key] = acc.get(key, 0.0) + wt
    keys = sorted(acc)
    return np.array(keys, dtype=np.int64).reshape(len(keys), d), np.array([acc[k] for k in keys])


def node_values(digits: np.ndarray, level: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """x = lo + (cos(pi c / D) + 1)(hi - lo) / 2 for every digit c."""
    D = digit_base(level)
    return lo + (np.cos(np.pi * np.asarray(digits, dtype=np.float64) / D) + 1.0) * (hi - lo) / 2.0


def sc_offline(nc: int, m: int, fam: dict, local_vars: list[list[int]], digits: np.ndarray, level: int,
               lo: float = -1.0, hi: float = 1.0) -> dict:
    """Dictionaries: per patch K the distinct local points (sorted) of the
    global points and S_K at each (plain cell solves, non-local variables 0)."""
    nxi = fam["g"] ** 2
    dicts = {}
    for K, lv in enumerate(local_vars):
        loc = sorted({tuple(int(v) for v in row) for row in digits[:, lv]}) if lv else [()]
        xs = np.zeros((len(loc), nxi))
        for r, key in enumerate(loc):
            for i, j in enumerate(lv):
                xs[r, j] = node_values(key[i], level, lo, hi)
        dicts[K] = (loc, ri.patch_S(xs, K, nc, m, fam))
    return dict(dicts=dicts, local_vars=local_vars, level=level, lo=lo, hi=hi)


def sc_plug_in(model: dict, digits: np.ndarray) -> np.ndarray:
    """Online search and plug-in: S [npts][M][10]."""
    M = len(model["local_vars"])
    S = np.zeros((digits.shape[0], M, 10))
    for K, lv in enumerate(model["local_vars"]):
        loc, tab = model["dicts"][K]
        where = {key: r for r, key in enumerate(loc)}
        for p in range(digits.shape[0]):
            S[p, K] = tab[where[tuple(int(v) for v in digits[p, lv])]]
    return S


def quadrature(U: np.ndarray, w: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """E ~ sum_p w_p U_p and var ~ sum_p w_p U_p^2 - E^2 (eq. sparseintegration
    and the variance formula after it)."""
    mean = np.einsum("p,pi->i", w, U)
    return mean, np.einsum("p,pi->i", w, U * U) - mean * mean


def sc_direct(nc: int, m: int, fam: dict, digits: np.ndarray, level: int, lo: float = -1.0,
              hi: float = 1.0) -> np.ndarray:
    """S [npts][M][10] by the plain path at every global collocation point
    (every variable at its node value): the definition the dictionaries must
    reproduce."""
    xi = node_values(digits, level, lo, hi)
    a = core.coef_bumps(xi, nc * m, fam["g"], fam["rho"], fam["eps"], fam["base"], fam["amp"], fam["beta"])
    S, st, _ = core.upscale(a, nc, nc, m)
    if np.any(st != 0):
        raise RuntimeError("plain solve failed at a collocation point")
    return S


# ---------------------------------------------------------------------------
# Sparse-grid interpolation of S_K in the local variables (Sec. 3.1 with the
# sparse node sets of Sec. 4.1.2 and Sec. 5.3): Smolyak's combination of tensor
# Lagrange interpolants on the nested Clenshaw-Curtis nodes,
#   I(L, k) f = sum over the terms of A(L, k) of c_i (U_i1 x ... x U_ik) f,
# U_i the one-dimensional Lagrange interpolant through the level-i nodes
# (level 1: the constant through the midpoint).  Its nodes are the points
# of the level-L sparse grid in k variables.
# ---------------------------------------------------------------------------
def level_nodes(i: int) -> np.ndarray:
    """The level-i nested Clenshaw-Curtis nodes on [-1, 1]: cos(pi j / (n-1))."""
    return cc_rule(i)[0]


def smolyak_interp(values: dict, k: int, level: int, t: np.ndarray) -> np.ndarray:
    """The Smolyak interpolant at the points t [N][k] (coordinates on
    [-1, 1]) of nodal values `values` {digits tuple: array [E]} on the
    level-`level` grid in k variables; [N][E]."""
    t = np.atleast_2d(np.asarray(t, dtype=np.float64))
    N = t.shape[0]
    D = digit_base(level)
    E = len(next(iter(values.values())))
    out = np.zeros((N, E))
    if k == 0:
        return out + values[()][None, :]
    for c, idx in smolyak_terms(k, level):
        bases = []
        digs = []
        for d, i in enumerate(idx):
            nodes = level_nodes(i)
            bases.append(ri.lagrange_basis(t[:, d], nodes) if len(nodes) > 1 else np.ones((N, 1)))
            n = len(nodes)
            digs.append([D // 2] if n == 1 else [j * D // (n - 1) for j in range(n)])
        for js in itertools.product(*[range(len(g)) for g in digs]):
            w = np.full(N, float(c))
            for d, j in enumerate(js):
                w = w * bases[d][:, j]
            out += w[:, None] * values[tuple(digs[d][j] for d, j in enumerate(js))][None, :]
    return out


def sgi_offline(nc: int, m: int, fam: dict, local_vars: list[list[int]], level: int, lo: float = -1.0,
                hi: float = 1.0) -> dict:
    """Per patch K with k local variables: S_K at the level-`level` sparse
    grid in k variables (plain cell solves, non-local variables 0)."""
    nxi = fam["g"] ** 2
    tables = {}
    for K, lv in enumerate(local_vars):
        dg, _ = sparse_grid(len(lv), level) if lv else (np.zeros((1, 0), dtype=np.int64), None)
        xs = np.zeros((len(dg), nxi))
        for i, j in enumerate(lv):
            xs[:, j] = node_values(dg[:, i], level, lo, hi)
        S = ri.patch_S(xs, K, nc, m, fam)
        tables[K] = {tuple(int(v) for v in row): S[r] for r, row in enumerate(dg)}
    return dict(tables=tables, local_vars=local_vars, level=level, lo=lo, hi=hi)


def sgi_online(model: dict, xi: np.ndarray, nc: int, m: int, fam: dict):
    """S [N][M][10] and the fallback mask [N][M]: the interpolant where every
    local variable lies in [lo, hi], the plain path elsewhere."""
    xi = np.atleast_2d(xi)
    N, M = xi.shape[0], nc * nc
    lo, hi = model["lo"], model["hi"]
    S = np.zeros((N, M, 10))
    fb = np.zeros((N, M), dtype=bool)
    for K in range(M):
        lv = model["local_vars"][K]
        x = xi[:, lv]
        inside = np.all((x >= lo) & (x <= hi), axis=1)
        if np.any(inside):
            t = 2.0 * (x[inside] - lo) / (hi - lo) - 1.0
            S[inside, K] = smolyak_interp(model["tables"][K], len(lv), model["level"], t)
        if np.any(~inside):
            S[~inside, K] = ri.patch_S(xi[~inside], K, nc, m, fam)
        fb[:, K] = ~inside
    return S, fb
