"""The short-correlation Gaussian medium of Sec. 5.3 and its local KL
parametrization (Sec. 2.1, eqs. domainpar, localCov, localKL,
local_KL_truncation).  Test infrastructure only (see package doc).

Medium.  kappa = 0.1 + exp(beta) (eq. mediaEx2), beta a centred Gaussian
field with covariance exp(-|x1-y1|^2/l1^2 - |x2-y2|^2/l2^2) (eq. betaCov).
Sampling by the randomized spectral method: with wave vectors w_j whose
components are N(0, 2/l^2) (the covariance is the characteristic function
of that normal law) and phases phi_j uniform on [0, 2 pi),
  beta(x) = sqrt(2/J) sum_j cos(w_j . x + phi_j),
which has exactly this covariance for any J and is Gaussian as J grows.
The draws come in as standard normals z and uniforms u: w_j = sqrt(2) (z_j1/l1,
z_j2/l2), phi_j = 2 pi u_j.  The field is taken at element centroids.

Local KL.  The patches are the coarse elements (non-overlapping, eq.
domainpar).  On the m x m centroids of a patch the discrete eigenproblem of
the covariance matrix C (dense, m^2 x m^2) with the L2 inner product h^2 sum
gives eigenvalues lambda = h^2 mu and modes f = v / h for the eigenpairs
(mu, v) of C (v of unit length), so that
  xi_k = (1/sqrt(lambda_k)) int (beta - 0) f_k = v_k . beta / sqrt(mu_k),
  beta ~ sum_{k <= K} sqrt(mu_k) xi_k v_k     (eqs. localKL, local_KL_truncation),
the KL being applied to the Gaussian field beta (kappa is non-affine in xi).
The covariance is translation invariant, so one set of modes serves every
patch; the same holds for the oversampled patches of Sec. 2.2 (side m + 2o,
moved inside the domain at its edge), the domains on which Sec. 5.3 takes the
local KL.  Outside the box |xi_k| <= 3 the interpolant is not used (the plain
path is); for independent standard normal xi_k the probability of that is
1 - P(|Z| <= 3)^K.
"""
from __future__ import annotations

from math import erf, sqrt

import numpy as np


def field(z: np.ndarray, u: np.ndarray, nfine: int, l1: float, l2: float) -> np.ndarray:
    """beta [N][nfine][nfine] (rows = y) at the element centroids."""
    N, J, _ = z.shape
    c = (np.arange(nfine) + 0.5) / nfine
    X, Y = np.meshgrid(c, c)
    out = np.zeros((N, nfine, nfine))
    for s in range(N):
        acc = np.zeros((nfine, nfine))
        for j in range(J):
            w1 = sqrt(2.0) * z[s, j, 0] / l1
            w2 = sqrt(2.0) * z[s, j, 1] / l2
            acc += np.cos(w1 * X + w2 * Y + 2.0 * np.pi * u[s, j])
        out[s] = sqrt(2.0 / J) * acc
    return out


def kappa(beta: np.ndarray) -> np.ndarray:
    return 0.1 + np.exp(beta)


def patch_covariance(m: int, h: float, l1: float, l2: float) -> np.ndarray:
    """Dense covariance of beta between the m^2 centroids of one patch
    (row-major: index = iy m + ix)."""
    c = (np.arange(m) + 0.5) * h
    X, Y = np.meshgrid(c, c)
    x, y = X.ravel(), Y.ravel()
    return np.exp(-((x[:, None] - x[None, :]) ** 2) / l1**2 - ((y[:, None] - y[None, :]) ** 2) / l2**2)


def local_kl(m: int, h: float, l1: float, l2: float, K: int):
    """(mu [K], V [K][m][m], captured fraction) of the K largest eigenpairs
    of the dense patch covariance (numpy eigh as the library step)."""
    C = patch_covariance(m, h, l1, l2)
    mu, V = np.linalg.eigh(C)
    order = np.argsort(mu)[::-1]
    mu, V = mu[order], V[:, order]
    return mu[:K], V[:, :K].T.reshape(K, m, m), float(mu[:K].sum() / mu.sum())


def project(beta: np.ndarray, nc: int, m: int, mu: np.ndarray, V: np.ndarray) -> np.ndarray:
    """xi [N][nc*nc][K] of every patch (element K = ky nc + kx)."""
    N = beta.shape[0]
    Kt = len(mu)
    xi = np.zeros((N, nc * nc, Kt))
    for ky in range(nc):
        for kx in range(nc):
            blk = beta[:, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m].reshape(N, -1)
            for k in range(Kt):
                xi[:, ky * nc + kx, k] = blk @ V[k].ravel() / np.sqrt(mu[k])
    return xi


def project_patches(beta: np.ndarray, nc: int, m: int, o: int, mu: np.ndarray, V: np.ndarray) -> np.ndarray:
    """xi [N][nc*nc][K] on the oversampled patches (Sec. 2.2: side m + 2o
    fine cells around each coarse element, moved inside the domain where it
    would stick out, so every patch has the same shape and one set of modes
    of side m + 2o serves all of them).  o = 0 gives project()."""
    N = beta.shape[0]
    nf = nc * m
    P = m + 2 * o
    if P > nf:
        raise ValueError("the oversampled patch is larger than the domain")
    Kt = len(mu)

    def origin(k):
        return min(max(k * m - o, 0), nf - P)

    xi = np.zeros((N, nc * nc, Kt))
    for ky in range(nc):
        for kx in range(nc):
            x0, y0 = origin(kx), origin(ky)
            blk = beta[:, y0:y0 + P, x0:x0 + P].reshape(N, -1)
            for k in range(Kt):
                xi[:, ky * nc + kx, k] = blk @ V[k].ravel() / np.sqrt(mu[k])
    return xi


def truncated_kappa_blocks(xi: np.ndarray, mu: np.ndarray, V: np.ndarray, K: int) -> np.ndarray:
    """kappa on every (sample, patch) from its first K local parameters:
    [N][P][m][m] = 0.1 + exp(sum_{k<K} sqrt(mu_k) xi_k V_k)."""
    b = np.einsum("npk,kij->npij", xi[:, :, :K] * np.sqrt(mu[:K]), V[:K])
    return 0.1 + np.exp(b)


def outside_probability(K: int, box: float = 3.0) -> float:
    """1 - P(|Z| <= box)^K for independent standard normals."""
    return 1.0 - erf(box / sqrt(2.0)) ** K


# ---------------------------------------------------------------------------
# Interpolation of S in the local KL parameters (Sec. 5.3 with Sec. 3.1):
# one table serves every coarse element (the covariance is translation
# invariant, so every element has the same modes): S at the tensor
# Chebyshev-Gauss-Lobatto nodes of [-box, box]^K, computed by the plain path
# on the truncated coefficient of each node; online, the tensor Lagrange
# interpolant at the pair's parameters, or the plain path on the sample's own
# kappa block when a parameter lies outside the box.
# ---------------------------------------------------------------------------
def kl_interp_offline(m: int, mu: np.ndarray, V: np.ndarray, nn: int, box: float = 3.0) -> dict:
    import itertools

    from . import core, ri

    K = len(mu)
    nodes = ri.cgl_nodes(nn, -box, box)
    xi_nodes = np.array([[nodes[d] for d in digits] for digits in itertools.product(range(nn), repeat=K)])
    blocks = truncated_kappa_blocks(xi_nodes[None], mu, V, K)[0]  # [nn^K][m][m]
    S, st, _ = core.upscale(blocks, 1, 1, m)
    if np.any(st != 0):
        raise RuntimeError("plain solve failed at a node")
    return dict(table=S[:, 0, :], nodes=nodes, box=box, K=K)


def kl_interp_online(model: dict, xi: np.ndarray, kap: np.ndarray, nc: int, m: int):
    """(S [N][nc*nc][10], fallback mask [N][nc*nc])."""
    from . import core, ri

    N, P, K = xi.shape
    box = model["box"]
    S = np.zeros((N, P, 10))
    fb = ~np.all(np.abs(xi) <= box, axis=2)
    for p in range(P):
        inside = ~fb[:, p]
        if np.any(inside):
            S[inside, p] = ri.ri_eval(model["table"], model["nodes"], xi[inside, p])
        if np.any(~inside):
            ky, kx = p // nc, p % nc
            blk = np.ascontiguousarray(kap[~inside, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m])
            Sp, _, _ = core.upscale(blk, 1, 1, m)
            S[~inside, p] = Sp[:, 0, :]
    return S, fb


# --- interpolation of the oversampled Petrov-Galerkin stiffness in the
# --- parameters of the oversampled patch (Secs. 2.2, 3.1 and 5.3)


def patch_origin(k: int, m: int, o: int, nf: int) -> int:
    """First fine cell (one axis) of the oversampled patch of element k."""
    return min(max(k * m - o, 0), nf - (m + 2 * o))


def element_class(k: int, m: int, o: int, nc: int) -> int:
    """Where element k sits in its patch along one axis: its offset from the
    patch origin is 0, o or 2o (for 1 <= o <= m), class 0, 1 or 2."""
    return (k * m - patch_origin(k, m, o, nc * m)) // o


def os_S_embedded(blocks: np.ndarray, m: int, o: int, cx: int, cy: int) -> np.ndarray:
    """[n][16] oversampled Petrov-Galerkin stiffness of an element at class
    (cx, cy) whose patch coefficient is blocks[i] ([n][m+2o][m+2o]): the
    patch placed in a 3 x 3-element mesh (where element (cx, cy) has that
    class; the rest of that mesh is 1 and is never read by the cell problems,
    which live on the patch), element (cx, cy) of it."""
    from . import core

    P, nf3 = m + 2 * o, 3 * m
    x0, y0 = patch_origin(cx, m, o, nf3), patch_origin(cy, m, o, nf3)
    out = np.zeros((len(blocks), 16))
    for i, blk in enumerate(blocks):
        f = np.ones((nf3, nf3))
        f[y0:y0 + P, x0:x0 + P] = blk
        out[i] = core.cell_S_os(f, m, o, cx, cy).ravel()
    return out


def kl_interp_os_offline(m: int, o: int, mu: np.ndarray, V: np.ndarray, nn: int, box: float = 3.0) -> dict:
    """Tables of the 16 entries at the nn^K Lobatto tensor nodes of the patch
    parameters, one per element class: at a node the patch coefficient is the
    truncated local KL 0.1 + exp(sum_k sqrt(mu_k) xi_k V_k) (side m + 2o)."""
    import itertools

    from . import ri

    if not 1 <= o <= m:
        raise ValueError("need 1 <= o <= m")
    K = len(mu)
    nodes = ri.cgl_nodes(nn, -box, box)
    xi_nodes = np.array([[nodes[d] for d in digits] for digits in itertools.product(range(nn), repeat=K)])
    blocks = truncated_kappa_blocks(xi_nodes[None], mu, V, K)[0]
    tables = {(cx, cy): os_S_embedded(blocks, m, o, cx, cy) for cy in range(3) for cx in range(3)}
    return dict(tables=tables, nodes=nodes, box=box, K=K, m=m, o=o)


def kl_sgi_os_offline(m: int, o: int, mu: np.ndarray, V: np.ndarray, level: int, box: float = 3.0) -> dict:
    """The same tables at the nodes of the level-`level` Smolyak sparse grid
    (nested Clenshaw-Curtis) in the K patch parameters on [-box, box]^K: the
    node set of the Chebyshev-Lobatto sparse-grid interpolation of Sec. 5.3."""
    from . import sc

    if not 1 <= o <= m:
        raise ValueError("need 1 <= o <= m")
    K = len(mu)
    dg, _ = sc.sparse_grid(K, level)
    xs = np.stack([sc.node_values(dg[:, i], level, -box, box) for i in range(K)], axis=1)
    blocks = truncated_kappa_blocks(xs[None], mu, V, K)[0]
    tables = {}
    for cy in range(3):
        for cx in range(3):
            S = os_S_embedded(blocks, m, o, cx, cy)
            tables[(cx, cy)] = {tuple(int(v) for v in row): S[r] for r, row in enumerate(dg)}
    return dict(tables=tables, level=level, box=box, K=K, m=m, o=o, sparse=True)


def kl_interp_os_online(model: dict, xi: np.ndarray, kap: np.ndarray, nc: int):
    """(S16 [N][nc*nc][16], fallback mask [N][nc*nc]) from the patch
    parameters xi [N][nc*nc][K]: inside the box the interpolant of the
    element's class table (tensor Lagrange, or Smolyak for a sparse-grid model), outside it the oversampled stiffness of the
    sample's own coefficient kap [N][nc m][nc m]."""
    from . import core, ri, sc

    m, o, box = model["m"], model["o"], model["box"]
    N, M, K = xi.shape
    S = np.zeros((N, M, 16))
    fb = ~np.all(np.abs(xi) <= box, axis=2)
    for p in range(M):
        kx, ky = p % nc, p // nc
        cls = (element_class(kx, m, o, nc), element_class(ky, m, o, nc))
        inside = ~fb[:, p]
        if np.any(inside):
            if model.get("sparse"):
                S[inside, p] = sc.smolyak_interp(model["tables"][cls], K, model["level"], xi[inside, p] / box)
            else:
                S[inside, p] = ri.ri_eval(model["tables"][cls], model["nodes"], xi[inside, p])
        for s in np.nonzero(~inside)[0]:
            S[s, p] = core.cell_S_os(kap[s], m, o, kx, ky).ravel()
    return S, fb
