"""ctypes binding of the C oracle (test infrastructure only; see package doc).

Every function takes and returns numpy float64 arrays.  The shared library is
built from ``stomsfem_oracle.c`` with plain gcc; ``build()`` compiles it and
``load()`` compiles it only when no built library is present.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "stomsfem_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

BC_LINEAR = 0
BC_OSC = 1
PACK = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]

_lib = None


def build() -> str:
    """Compile the oracle (gcc -O3 for x86-64-v3, OpenMP).  Always recompiles.

    x86-64-v3 (AVX2, FMA) rather than -march=native: the library is built in
    one place and also loaded on other hosts.  ISO C mode keeps floating-point
    contraction off, so FMA instructions do not change the results."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", SRC,
           "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = C.CDLL(LIB)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    i64, i32, dbl, sz = C.c_int64, C.c_int, C.c_double, C.c_ssize_t
    sig = {
        "orc_q1_kref": (None, [dp]),
        "orc_band_chol": (i32, [i32, i32, dp]),
        "orc_band_solve": (None, [i32, i32, dp, i32, dp]),
        "orc_cell_phi": (i32, [i32, dp, sz, i32, dp]),
        "orc_energy_S": (None, [i32, dp, sz, dp, dp, dp]),
        "orc_galerkin_load": (None, [i32, dbl, dbl, dp, dp]),
        "orc_cell_S": (i32, [i32, dp, sz, i32, dp, dp]),
        "orc_upscale": (i32, [i64, i32, i32, i32, dp, i32, dp, ip, dp, i32]),
        "orc_coarse_one": (i32, [i32, i32, dp, dp, dp]),
        "orc_coarse_solve": (i32, [i32, i32, i64, dp, dp, dp, dp, dp, ip, i32]),
        "orc_fine_fem": (i32, [i32, dp, dbl, dp]),
        "orc_cell_system_dense": (i32, [i32, dp, sz, i32, dp, dp]),
        "orc_coef_bumps": (i32, [i64, i32, dp, i32, i32, dbl, dbl, dbl, dbl, dbl, dp, i32]),
        "orc_coef_features": (i32, [i64, i32, i32, ip, dp, dp, dp, dp, i32, dbl, dp, i32]),
        "orc_os_origin": (i32, [i32, i32, i32, i32]),
        "orc_cell_phi_os": (i32, [i32, i32, i32, i32, dp, sz, i32, i32, dp, dp]),
        "orc_cell_S_os": (i32, [i32, i32, i32, i32, dp, sz, i32, i32, dp]),
        "orc_upscale_os": (i32, [i64, i32, i32, i32, i32, dp, dp, ip, i32]),
        "orc_band_lu_solve": (i32, [i32, i32, i32, dp, dp]),
        "orc_coarse_pg_solve": (i32, [i32, i32, i64, dp, dp, dp, dp, dp, ip, i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(x):
    if x is None:
        return None
    assert x.dtype == np.float64 and x.flags["C_CONTIGUOUS"]
    return x.ctypes.data_as(C.POINTER(C.c_double))


def _c(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def q1_kref() -> np.ndarray:
    K = np.zeros(16)
    load().orc_q1_kref(_p(K))
    return K.reshape(4, 4)


def band_chol(B: np.ndarray) -> tuple[np.ndarray, int]:
    """B: [n][bw+1] lower band (B[i,d] = A[i,i-d]).  Returns (L band, status)."""
    B = _c(B).copy()
    n, w = B.shape
    st = load().orc_band_chol(n, w - 1, _p(B))
    return B, st


def band_solve(L: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    L = _c(L)
    x = _c(np.atleast_2d(rhs)).copy()
    n, w = L.shape
    load().orc_band_solve(n, w - 1, _p(L), x.shape[0], _p(x))
    return x


def cell_phi(a_blk: np.ndarray, bc: int = BC_LINEAR) -> np.ndarray:
    """Four cell-problem solutions on the (m+1)^2 node grid: [4][m+1][m+1]."""
    a_blk = _c(a_blk)
    m = a_blk.shape[0]
    phi = np.zeros((4, m + 1, m + 1))
    st = load().orc_cell_phi(m, _p(a_blk), a_blk.shape[1], bc, _p(phi))
    if st != 0:
        raise RuntimeError(f"orc_cell_phi status {st}")
    return phi


def energy_S(a_blk: np.ndarray, phi: np.ndarray, test: np.ndarray | None = None) -> np.ndarray:
    a_blk = _c(a_blk)
    m = a_blk.shape[0]
    S = np.zeros(16)
    load().orc_energy_S(m, _p(a_blk), a_blk.shape[1], _p(_c(phi)), _p(None if test is None else _c(test)), _p(S))
    return S.reshape(4, 4)


def galerkin_load(phi: np.ndarray, H: float, f: float = 1.0) -> np.ndarray:
    phi = _c(phi)
    m = phi.shape[1] - 1
    b = np.zeros(4)
    load().orc_galerkin_load(m, H, f, _p(phi), _p(b))
    return b


def cell_S(a_blk: np.ndarray, bc: int = BC_LINEAR) -> tuple[np.ndarray, float]:
    """Packed upscaled stiffness [10] and the partition-of-unity defect."""
    a_blk = _c(a_blk)
    m = a_blk.shape[0]
    out = np.zeros(10)
    pu = C.c_double(0.0)
    st = load().orc_cell_S(m, _p(a_blk), a_blk.shape[1], bc, _p(out), C.byref(pu))
    if st != 0:
        raise RuntimeError(f"orc_cell_S status {st}")
    return out, pu.value


def unpack(Sp: np.ndarray) -> np.ndarray:
    """[..., 10] packed -> [..., 4, 4] symmetric."""
    Sp = np.asarray(Sp)
    out = np.zeros(Sp.shape[:-1] + (4, 4))
    for q, (i, j) in enumerate(PACK):
        out[..., i, j] = Sp[..., q]
        out[..., j, i] = Sp[..., q]
    return out


def pack(S4: np.ndarray) -> np.ndarray:
    S4 = np.asarray(S4)
    return np.stack([S4[..., i, j] for (i, j) in PACK], axis=-1)


def upscale(a: np.ndarray, ncx: int, ncy: int, m: int, bc: int = BC_LINEAR, nthreads: int = 0):
    """a: [N][ncy*m][ncx*m] -> (S [N][M][10], status [N][M], max PU defect)."""
    a = _c(a)
    N = a.shape[0]
    assert a.shape[1:] == (ncy * m, ncx * m)
    S = np.zeros((N, ncx * ncy, 10))
    status = np.zeros((N, ncx * ncy), dtype=np.int32)
    pu = C.c_double(0.0)
    st = load().orc_upscale(N, ncx, ncy, m, _p(a), bc, _p(S), status.ctypes.data_as(C.POINTER(C.c_int32)),
                            C.byref(pu), nthreads)
    if st != 0:
        raise RuntimeError(f"orc_upscale status {st}")
    return S, status, pu.value


def coarse_solve(S: np.ndarray, ncx: int, ncy: int, load_vec: np.ndarray | None = None, nthreads: int = 0):
    """S: [N][M][10] -> (U [N][(ncx-1)(ncy-1)], mean, var)."""
    S = _c(S)
    N = S.shape[0]
    nU = (ncx - 1) * (ncy - 1)
    U = np.zeros((N, nU))
    mean = np.zeros(nU)
    var = np.zeros(nU)
    status = np.zeros(N, dtype=np.int32)
    lv = None if load_vec is None else _c(load_vec)
    st = load().orc_coarse_solve(ncx, ncy, N, _p(S), _p(lv), _p(U), _p(mean), _p(var),
                                 status.ctypes.data_as(C.POINTER(C.c_int32)), nthreads)
    if st != 0:
        raise RuntimeError(f"orc_coarse_solve status {st}")
    return U, mean, var


def fine_fem(a: np.ndarray, f: float = 1.0) -> np.ndarray:
    """Global Q1 FEM on the nf x nf grid: interior nodal values [(nf-1)^2]."""
    a = _c(a)
    nf = a.shape[0]
    u = np.zeros((nf - 1) * (nf - 1))
    st = load().orc_fine_fem(nf, _p(a), f, _p(u))
    if st != 0:
        raise RuntimeError(f"orc_fine_fem status {st}")
    return u


def cell_system_dense(a_blk: np.ndarray, bc: int = BC_LINEAR):
    """(K_II [nI][nI], lifts [4][nI]) with lift^l = -K_IB g^l."""
    a_blk = _c(a_blk)
    m = a_blk.shape[0]
    nI = (m - 1) ** 2
    K = np.zeros((nI, nI))
    lift = np.zeros((4, nI))
    load().orc_cell_system_dense(m, _p(a_blk), a_blk.shape[1], bc, _p(K), _p(lift))
    return K, lift


def coef_bumps(xi: np.ndarray, nfine: int, g: int, rho: float, eps: float,
               base: float = 2.0, amp: float = 1.8, beta: float = 0.5, nthreads: int = 0) -> np.ndarray:
    """Coefficient samples a[N][nfine][nfine] of the bump/checkerboard family."""
    xi = _c(xi)
    N, nxi = xi.shape
    a = np.zeros((N, nfine, nfine))
    st = load().orc_coef_bumps(N, nfine, _p(xi), nxi, g, rho, eps, base, amp, beta, _p(a), nthreads)
    if st != 0:
        raise RuntimeError(f"orc_coef_bumps status {st}")
    return a


def coef_features(xi: np.ndarray, nfine: int, kind, x0, y0, size, decades: float = 4.0,
                  nthreads: int = 0) -> np.ndarray:
    """Coefficient samples a[N][nfine][nfine] of the channels-and-inclusions
    medium (see orc_coef_features)."""
    xi = _c(xi)
    N, nxi = xi.shape
    kind = np.ascontiguousarray(kind, dtype=np.int32)
    x0, y0, size = _c(x0), _c(y0), _c(size)
    a = np.zeros((N, nfine, nfine))
    st = load().orc_coef_features(N, nfine, len(kind), kind.ctypes.data_as(C.POINTER(C.c_int32)), _p(x0), _p(y0),
                                  _p(size), _p(xi), nxi, decades, _p(a), nthreads)
    if st != 0:
        raise RuntimeError(f"orc_coef_features status {st}")
    return a


# --- oversampling and the Petrov-Galerkin local stiffness --------------------


def os_origin(k: int, m: int, o: int, nf: int) -> int:
    """First fine cell (one axis) of the oversampled patch of coarse element k."""
    return int(load().orc_os_origin(k, m, o, nf))


def cell_phi_os(a: np.ndarray, m: int, o: int, kx: int, ky: int):
    """Oversampled basis on K: (phi [4][m+1][m+1], Psi [4][4] = psi^j(x_k)).
    a: one sample's whole field [nfy][nfx]."""
    a = _c(a)
    phi = np.zeros((4, m + 1, m + 1))
    Psi = np.zeros((4, 4))
    st = load().orc_cell_phi_os(m, o, a.shape[1], a.shape[0], _p(a), a.shape[1], kx, ky, _p(phi), _p(Psi))
    if st != 0:
        raise RuntimeError(f"orc_cell_phi_os status {st}")
    return phi, Psi


def cell_S_os(a: np.ndarray, m: int, o: int, kx: int, ky: int) -> np.ndarray:
    """Petrov-Galerkin stiffness S[l][l'] (trial l, bilinear test l') of element (kx, ky)."""
    a = _c(a)
    S = np.zeros(16)
    st = load().orc_cell_S_os(m, o, a.shape[1], a.shape[0], _p(a), a.shape[1], kx, ky, _p(S))
    if st != 0:
        raise RuntimeError(f"orc_cell_S_os status {st}")
    return S.reshape(4, 4)


def upscale_os(a: np.ndarray, ncx: int, ncy: int, m: int, o: int, nthreads: int = 0):
    """a: [N][ncy*m][ncx*m] -> (S16 [N][M][16] row-major [l][l'], status [N][M])."""
    a = _c(a)
    N = a.shape[0]
    assert a.shape[1:] == (ncy * m, ncx * m)
    S = np.zeros((N, ncx * ncy, 16))
    status = np.zeros((N, ncx * ncy), dtype=np.int32)
    st = load().orc_upscale_os(N, ncx, ncy, m, o, _p(a), _p(S), status.ctypes.data_as(C.POINTER(C.c_int32)),
                               nthreads)
    if st != 0:
        raise RuntimeError(f"orc_upscale_os status {st}")
    return S, status


def band_lu_solve(A: np.ndarray, b: np.ndarray, kl: int, ku: int) -> np.ndarray:
    """Solve the dense-stored banded A x = b with the oracle's banded LU."""
    A = _c(A)
    n = A.shape[0]
    w = 2 * kl + ku + 1
    W = np.zeros((n, w))
    for i in range(n):
        for c in range(max(0, i - kl), min(n, i + ku + 1)):
            W[i, c - i + kl] = A[i, c]
    x = _c(b).copy()
    st = load().orc_band_lu_solve(n, kl, ku, _p(W), _p(x))
    if st != 0:
        raise RuntimeError(f"orc_band_lu_solve status {st}")
    return x


def coarse_solve_pg(S16: np.ndarray, ncx: int, ncy: int, load_vec: np.ndarray | None = None, nthreads: int = 0):
    """S16: [N][M][16] -> (U [N][(ncx-1)(ncy-1)], mean, var) of the Petrov-Galerkin coarse system."""
    S16 = _c(S16)
    N = S16.shape[0]
    nU = (ncx - 1) * (ncy - 1)
    U = np.zeros((N, nU))
    mean = np.zeros(nU)
    var = np.zeros(nU)
    status = np.zeros(N, dtype=np.int32)
    lv = None if load_vec is None else _c(load_vec)
    st = load().orc_coarse_pg_solve(ncx, ncy, N, _p(S16), _p(lv), _p(U), _p(mean), _p(var),
                                    status.ctypes.data_as(C.POINTER(C.c_int32)), nthreads)
    if st != 0:
        raise RuntimeError(f"orc_coarse_pg_solve status {st}")
    return U, mean, var
