"""Thin ctypes binding of libstomsfem.so with the C entry-point names.

Only argument marshalling happens here: torch tensors supply device memory and
the current HIP stream; every step of the computation runs in the library's
kernels.  There is no CPU fallback: if the library is missing or the tensors
are not on the GPU, the call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libstomsfem.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSPD, ENOCONV, EVERSION = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
PREC_F64, PREC_F32_REFINE64, PREC_BF16, PREC_AUTO, PREC_F32, PREC_F16 = 0, 1, 2, 3, 4, 5
MLP_NPARAM = 9940
MLP_BATCH = 32
MLP_KIN = 4
BC_LINEAR, BC_OSCILLATORY = 0, 1

_DT = {torch.float64: F64, torch.float32: F32}


class StomsfemError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


class BumpFamily(C.Structure):
    _fields_ = [("g", C.c_int32), ("rho", C.c_double), ("eps", C.c_double), ("base", C.c_double),
                ("amp", C.c_double), ("beta", C.c_double)]


class Stage(C.Structure):
    _fields_ = [("ncx", C.c_int32), ("ncy", C.c_int32), ("m", C.c_int32), ("nsamples", C.c_int64),
                ("a_dtype", C.c_int32), ("family", C.c_int32), ("bumps", BumpFamily),
                ("feature_map", C.c_void_p), ("nfeat", C.c_int32), ("decades", C.c_double),
                ("xi", C.c_void_p), ("nxi", C.c_int32), ("U", C.c_void_p), ("qoi_mean", C.c_void_p),
                ("qoi_var", C.c_void_p), ("status", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("m", C.c_int32), ("a_dtype", C.c_int32), ("lane_block", C.c_int32), ("tiled_waves", C.c_int32),
                ("precision", C.c_int32), ("candidates", C.c_int32), ("ms_default", C.c_double),
                ("ms_best", C.c_double)]


class Batch(C.Structure):
    _fields_ = [
        ("ncx", C.c_int32),
        ("ncy", C.c_int32),
        ("m", C.c_int32),
        ("a_dtype", C.c_int32),
        ("nsamples", C.c_int64),
        ("a", C.c_void_p),
        ("S", C.c_void_p),
        ("status", C.c_void_p),
    ]


_lib = None


def lib():
    """Load libstomsfem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python paper_1607_00693_amd/build.py` "
            "(or __graft_entry__.build()); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "stomsfem_version": (C.c_int, []),
        "stomsfem_last_error": (C.c_char_p, []),
        "stomsfem_coef_bumps": (C.c_int, [i64, i32, vp, i32, i32, dbl, dbl, dbl, dbl, dbl, vp, i32, vp]),
        "stomsfem_upscale": (C.c_int, [C.POINTER(Batch), i32, i32, i32, vp]),
        "stomsfem_upscale_reference": (C.c_int, [C.POINTER(Batch), i32, vp]),
        "stomsfem_upscale_queue": (C.c_int, [C.POINTER(Batch), i32, vp]),
        "stomsfem_element_loads": (C.c_int, [i32, i32, C.POINTER(dbl), vp, vp]),
        "stomsfem_coarse_solve": (C.c_int, [i32, i32, i64, vp, vp, vp, vp, vp, vp, vp]),
        "stomsfem_coarse_solve_pg": (C.c_int, [i32, i32, i64, vp, vp, vp, vp, vp, vp, vp]),
        "stomsfem_upscale_os": (C.c_int, [vp, i32, vp]),
        "stomsfem_workspace_reserve": (C.c_int, [i64]),
        "stomsfem_reduce": (C.c_int, [C.POINTER(Batch), i32, dbl, C.POINTER(vp), vp]),
        "stomsfem_reduce_apply": (C.c_int, [vp, C.POINTER(Batch), i32, vp]),
        "stomsfem_reduce_os": (C.c_int, [C.POINTER(Batch), i32, i32, dbl, C.POINTER(vp), vp]),
        "stomsfem_reduce_os_apply": (C.c_int, [vp, C.POINTER(Batch), i32, vp]),
        "stomsfem_model_export": (C.c_int, [vp, i32, vp, i64]),
        "stomsfem_model_free": (C.c_int, [vp]),
        "stomsfem_local_vars_bumps": (C.c_int, [i32, i32, i32, C.POINTER(BumpFamily), i32, vp, vp]),
        "stomsfem_mlp_create": (C.c_int, [i32, i32, i32, vp, vp, C.POINTER(BumpFamily), dbl, C.POINTER(vp)]),
        "stomsfem_local_vars_features": (C.c_int, [i32, i32, i32, vp, i32, i32, vp, vp]),
        "stomsfem_mlp_create_features": (C.c_int, [i32, i32, vp, i32, dbl, vp, dbl, C.POINTER(vp)]),
        "stomsfem_mlp_set_data": (C.c_int, [vp, vp, i32, vp, i64, vp]),
        "stomsfem_mlp_train": (C.c_int, [vp, i32, C.c_float, vp, vp, vp]),
        "stomsfem_mlp_grad": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "stomsfem_mlp_params": (C.c_int, [vp, vp, vp, vp]),
        "stomsfem_mlp_standardization": (C.c_int, [vp, vp, vp]),
        "stomsfem_mlp_predict": (C.c_int, [vp, vp, i32, i64, vp, i32, vp]),
        "stomsfem_mlp_gate": (C.c_int, [vp, vp, vp, i32, i64, dbl, vp, vp, vp, vp]),
        "stomsfem_coarse_solve_noalloc": (C.c_int, [i32, i32, i64, vp, vp, vp, vp, vp, vp, vp]),
        "stomsfem_fine_solve_pcg": (C.c_int, [vp, i32, i64, dbl, i32, vp, vp, vp, vp]),
        "stomsfem_upscale_surrogate": (C.c_int, [vp, vp, i32, i64, vp, vp, dbl, i32, vp, vp]),
        "stomsfem_workspace_release": (C.c_int, []),
        "stomsfem_feature_map": (C.c_int, [i32, i32, vp, vp, vp, vp, vp, vp]),
        "stomsfem_coef_features": (C.c_int, [i64, i32, vp, i32, vp, i32, dbl, vp, i32, vp]),
        "stomsfem_plan_create": (C.c_int, [C.POINTER(Stage), i32, C.POINTER(vp)]),
        "stomsfem_plan_launch": (C.c_int, [vp, i32, vp]),
        "stomsfem_plan_free": (C.c_int, [vp]),
        "stomsfem_autotune": (C.c_int, [C.POINTER(Batch), i32, C.POINTER(Tuning), vp]),
        "stomsfem_tuning_reset": (C.c_int, []),
        "stomsfem_model_save": (C.c_int, [vp, C.c_char_p]),
        "stomsfem_model_load": (C.c_int, [C.c_char_p, C.POINTER(vp)]),
        "stomsfem_model_shape": (C.c_int, [vp, vp, vp, vp, vp]),
        "stomsfem_stats_get": (C.c_int, [vp]),
        "stomsfem_stats_reset": (C.c_int, []),
        "stomsfem_surrogate_train": (C.c_int, [vp, i32, C.c_float, vp, vp, vp]),
        "stomsfem_interp_build": (C.c_int, [i32, i32, i32, vp, C.POINTER(BumpFamily), i32, dbl, dbl,
                                            C.POINTER(vp), vp]),
        "stomsfem_interp_apply": (C.c_int, [vp, vp, i32, i64, vp, vp, C.POINTER(i64), vp]),
        "stomsfem_sparse_grid": (C.c_int, [i32, i32, i64, C.POINTER(i64), vp, vp]),
        "stomsfem_sc_build": (C.c_int, [i32, i32, i32, vp, C.POINTER(BumpFamily), i32, dbl, dbl, vp, i64,
                                        C.POINTER(vp), vp]),
        "stomsfem_sc_apply": (C.c_int, [vp, vp, i32, i64, vp, vp, vp]),
        "stomsfem_quadrature": (C.c_int, [vp, vp, i64, i32, vp, vp, vp]),
        "stomsfem_sgi_build": (C.c_int, [i32, i32, i32, vp, C.POINTER(BumpFamily), i32, dbl, dbl, C.POINTER(vp),
                                         vp]),
        "stomsfem_sgi_apply": (C.c_int, [vp, vp, i32, i64, vp, vp, C.POINTER(i64), vp]),
        "stomsfem_fine_solve": (C.c_int, [vp, i32, i64, vp, vp, vp]),
        "stomsfem_two_level_mc": (C.c_int, [vp, i64, vp, vp, i64, i32, i32, vp, vp, vp, vp]),
        "stomsfem_coef_gauss": (C.c_int, [i64, i32, i32, vp, vp, dbl, dbl, vp, vp, vp]),
        "stomsfem_local_kl": (C.c_int, [i32, dbl, dbl, dbl, i32, vp, vp, vp]),
        "stomsfem_kl_project": (C.c_int, [i64, i32, i32, vp, i32, vp, vp, dbl, vp, vp, vp, vp]),
        "stomsfem_kl_project_patches": (C.c_int, [i64, i32, i32, i32, vp, i32, vp, vp, dbl, vp, vp, vp, vp]),
        "stomsfem_kl_blocks": (C.c_int, [i64, i32, i32, i32, vp, vp, vp, vp, vp]),
        "stomsfem_kl_interp_build": (C.c_int, [i32, i32, i32, i32, vp, vp, i32, dbl, C.POINTER(vp), vp]),
        "stomsfem_kl_interp_os_build": (C.c_int, [i32, i32, i32, i32, i32, vp, vp, i32, dbl, C.POINTER(vp), vp]),
        "stomsfem_kl_sgi_os_build": (C.c_int, [i32, i32, i32, i32, i32, vp, vp, i32, dbl, C.POINTER(vp), vp]),
        "stomsfem_kl_interp_apply": (C.c_int, [vp, vp, vp, i64, vp, vp, C.POINTER(i64), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(fn: str, rc: int):
    if rc != OK:
        msg = lib().stomsfem_last_error()
        raise StomsfemError(fn, rc, msg.decode() if msg else "")


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def version() -> int:
    return lib().stomsfem_version()


def coef_bumps(xi: torch.Tensor, nfine: int, g: int, rho: float, eps: float, base: float = 2.0,
               amp: float = 1.8, beta: float = 0.5, dtype=torch.float64, out: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    """Coefficient samples a[N][nfine][nfine] of the bump family (see stomsfem.h)."""
    assert xi.dtype == torch.float64
    N, nxi = xi.shape
    if out is None:
        out = torch.empty((N, nfine, nfine), dtype=dtype, device=xi.device)
    _check("stomsfem_coef_bumps", lib().stomsfem_coef_bumps(
        N, nfine, _ptr(xi), nxi, g, rho, eps, base, amp, beta, _ptr(out), _DT[out.dtype], _stream(stream)))
    return out


def make_batch(a: torch.Tensor, ncx: int, ncy: int, m: int, S: torch.Tensor, status: torch.Tensor | None,
               entries: int = 10) -> Batch:
    N = a.shape[0]
    assert a.shape[1:] == (ncy * m, ncx * m), f"a has shape {tuple(a.shape)}"
    assert S.dtype == torch.float64 and S.shape == (N, ncx * ncy, entries)
    if status is not None:
        assert status.dtype == torch.int32 and status.shape == (N, ncx * ncy)
    return Batch(ncx, ncy, m, _DT[a.dtype], N, _ptr(a), _ptr(S), _ptr(status))


def upscale(a: torch.Tensor, ncx: int, ncy: int, m: int, S: torch.Tensor | None = None,
            status: torch.Tensor | None = None, precision: int = PREC_F64, stream=None, bc: int = BC_LINEAR):
    """Upscaled stiffness S[N][ncy*ncx][10] for one homogeneous batch."""
    N = a.shape[0]
    if S is None:
        S = torch.empty((N, ncx * ncy, 10), dtype=torch.float64, device=a.device)
    b = make_batch(a, ncx, ncy, m, S, status)
    _check("stomsfem_upscale", lib().stomsfem_upscale(C.byref(b), 1, precision, bc, _stream(stream)))
    return S


def upscale_batches(batches: list[Batch], precision: int = PREC_F64, stream=None):
    arr = (Batch * len(batches))(*batches)
    _check("stomsfem_upscale", lib().stomsfem_upscale(arr, len(batches), precision, BC_LINEAR, _stream(stream)))


def upscale_queue(batches: list[Batch], stream=None):
    """One persistent launch over batches of m in {8, 16, 32}."""
    arr = (Batch * len(batches))(*batches)
    _check("stomsfem_upscale_queue", lib().stomsfem_upscale_queue(arr, len(batches), _stream(stream)))


def upscale_reference(a: torch.Tensor, ncx: int, ncy: int, m: int, S: torch.Tensor | None = None,
                      status: torch.Tensor | None = None, stream=None, bc: int = BC_LINEAR):
    N = a.shape[0]
    if S is None:
        S = torch.empty((N, ncx * ncy, 10), dtype=torch.float64, device=a.device)
    b = make_batch(a, ncx, ncy, m, S, status)
    _check("stomsfem_upscale_reference", lib().stomsfem_upscale_reference(C.byref(b), bc, _stream(stream)))
    return S


def element_loads(ncx: int, ncy: int, f=(2.0, 0.0, 0.0, 1.0), stream=None) -> torch.Tensor:
    """Element loads [ncy*ncx][4] of the bilinear source f[0] + f[1] x + f[2] y + f[3] x y
    (default: Sec. 5.3's 2 + x1 x2)."""
    fa = (C.c_double * 4)(*[float(v) for v in f])
    out = torch.empty((ncy * ncx, 4), dtype=torch.float64, device="cuda")
    _check("stomsfem_element_loads", lib().stomsfem_element_loads(ncx, ncy, fa, _ptr(out), _stream(stream)))
    return out


def coarse_solve(S: torch.Tensor, ncx: int, ncy: int, load: torch.Tensor | None = None,
                 U: torch.Tensor | None = None, qoi_mean: torch.Tensor | None = None,
                 qoi_var: torch.Tensor | None = None, status: torch.Tensor | None = None, stream=None):
    """Per-sample coarse solutions U[N][(ncx-1)(ncy-1)] and the MC mean/variance."""
    N = S.shape[0]
    assert S.dtype == torch.float64 and S.shape == (N, ncx * ncy, 10)
    nU = (ncx - 1) * (ncy - 1)
    dev = S.device
    if U is None:
        U = torch.empty((N, nU), dtype=torch.float64, device=dev)
    if qoi_mean is None:
        qoi_mean = torch.empty(nU, dtype=torch.float64, device=dev)
    if qoi_var is None:
        qoi_var = torch.empty(nU, dtype=torch.float64, device=dev)
    if load is not None:
        assert load.dtype == torch.float64 and load.shape == (ncx * ncy, 4)
    _check("stomsfem_coarse_solve", lib().stomsfem_coarse_solve(
        ncx, ncy, N, _ptr(S), _ptr(load), _ptr(U), _ptr(qoi_mean), _ptr(qoi_var), _ptr(status), _stream(stream)))
    return U, qoi_mean, qoi_var


def coef_gauss(z: torch.Tensor, u: torch.Tensor, nfine: int, l1: float, l2: float, with_beta: bool = False,
               stream=None):
    """Gaussian medium kappa[N][nfine][nfine] (and beta if asked) from the
    spectral draws z[N][J][2], u[N][J]."""
    assert z.dtype == torch.float64 and u.dtype == torch.float64 and z.is_contiguous() and u.is_contiguous()
    N, J = u.shape
    kappa = torch.empty((N, nfine, nfine), dtype=torch.float64, device=z.device)
    beta = torch.empty_like(kappa) if with_beta else None
    _check("stomsfem_coef_gauss", lib().stomsfem_coef_gauss(N, nfine, J, _ptr(z), _ptr(u), l1, l2, _ptr(beta),
                                                           _ptr(kappa), _stream(stream)))
    return (kappa, beta) if with_beta else kappa


def local_kl(m: int, h: float, l1: float, l2: float, K: int):
    """Host local KL of one coarse element: (mu [K], modes [K][m][m], captured)."""
    import numpy as np

    mu = np.zeros(K)
    modes = np.zeros((K, m, m))
    cap = C.c_double(0.0)
    _check("stomsfem_local_kl", lib().stomsfem_local_kl(m, h, l1, l2, K, mu.ctypes.data_as(C.c_void_p),
                                                       modes.ctypes.data_as(C.c_void_p), C.byref(cap)))
    return mu, modes, cap.value


def kl_project(beta: torch.Tensor, nc: int, m: int, mu: torch.Tensor, modes: torch.Tensor, box: float = 3.0,
               stream=None, oversample: int = 0):
    """(xi [N][nc*nc][K], outside [N][nc*nc] int32, number of outside pairs).
    oversample > 0: on the oversampled patches of side m + 2 oversample
    (modes of that side)."""
    N = beta.shape[0]
    K = mu.shape[0]
    xi = torch.empty((N, nc * nc, K), dtype=torch.float64, device=beta.device)
    outside = torch.empty((N, nc * nc), dtype=torch.int32, device=beta.device)
    count = torch.zeros(1, dtype=torch.int64, device=beta.device)
    if oversample == 0:
        _check("stomsfem_kl_project", lib().stomsfem_kl_project(N, nc, m, _ptr(beta), K, _ptr(mu), _ptr(modes), box,
                                                               _ptr(xi), _ptr(outside), _ptr(count), _stream(stream)))
    else:
        _check("stomsfem_kl_project_patches",
               lib().stomsfem_kl_project_patches(N, nc, m, oversample, _ptr(beta), K, _ptr(mu), _ptr(modes), box,
                                                 _ptr(xi), _ptr(outside), _ptr(count), _stream(stream)))
    return xi, outside, count


def kl_blocks(xi: torch.Tensor, mu: torch.Tensor, modes: torch.Tensor, Kuse: int, stream=None) -> torch.Tensor:
    """Truncated-KL coefficient blocks [npairs][m][m] for xi [..][K]."""
    K = mu.shape[0]
    m = modes.shape[-1]
    x = xi.reshape(-1, K)
    blocks = torch.empty((x.shape[0], m, m), dtype=torch.float64, device=xi.device)
    _check("stomsfem_kl_blocks", lib().stomsfem_kl_blocks(x.shape[0], m, Kuse, K, _ptr(x), _ptr(mu), _ptr(modes),
                                                         _ptr(blocks), _stream(stream)))
    return blocks


def kl_interp_build(ncx: int, ncy: int, m: int, mu: torch.Tensor, modes: torch.Tensor, nnodes: int,
                    box: float = 3.0, stream=None, oversample: int = 0, level: int | None = None) -> Model:
    """Offline: S at the tensor Lobatto nodes of the local KL parameters (one
    table for all elements); oversample > 0: the oversampled Petrov-Galerkin
    stiffness (16 entries) in the parameters of the oversampled patches (modes
    of side m + 2 oversample), one table per element class; with `level`, at
    the nodes of that sparse grid instead (nnodes is then unused)."""
    h = C.c_void_p()
    if level is not None:
        if oversample < 1:
            raise ValueError("the sparse-grid tables are for the oversampled stiffness (oversample >= 1)")
        _check("stomsfem_kl_sgi_os_build", lib().stomsfem_kl_sgi_os_build(
            ncx, ncy, m, oversample, mu.shape[0], _ptr(mu), _ptr(modes), level, box, C.byref(h), _stream(stream)))
    elif oversample == 0:
        _check("stomsfem_kl_interp_build", lib().stomsfem_kl_interp_build(
            ncx, ncy, m, mu.shape[0], _ptr(mu), _ptr(modes), nnodes, box, C.byref(h), _stream(stream)))
    else:
        _check("stomsfem_kl_interp_os_build", lib().stomsfem_kl_interp_os_build(
            ncx, ncy, m, oversample, mu.shape[0], _ptr(mu), _ptr(modes), nnodes, box, C.byref(h), _stream(stream)))
    md = Model(h, ncx, ncy, m)
    md.entries = 16 if oversample else 10
    return md


def kl_interp_apply(model: Model, xi: torch.Tensor, kappa: torch.Tensor, S: torch.Tensor | None = None,
                    status: torch.Tensor | None = None, stream=None):
    """Online: (S [N][M][10] (16 for an oversampled model), number of pairs
    computed from kappa)."""
    N = xi.shape[0]
    if S is None:
        S = torch.empty((N, model.ncx * model.ncy, getattr(model, "entries", 10)), dtype=torch.float64,
                        device=xi.device)
    nfb = C.c_int64(0)
    _check("stomsfem_kl_interp_apply", lib().stomsfem_kl_interp_apply(
        model.handle, _ptr(xi), _ptr(kappa), N, _ptr(S), _ptr(status), C.byref(nfb), _stream(stream)))
    return S, nfb.value


def fine_solve(a: torch.Tensor, u: torch.Tensor | None = None, status: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    """Fine-grid FEM solutions u[N][(nfine-1)^2] for a[N][nfine][nfine] (FP64)."""
    assert a.dtype == torch.float64 and a.is_contiguous() and a.shape[1] == a.shape[2]
    N, nf = a.shape[0], a.shape[1]
    if u is None:
        u = torch.empty((N, (nf - 1) ** 2), dtype=torch.float64, device=a.device)
    _check("stomsfem_fine_solve", lib().stomsfem_fine_solve(_ptr(a), nf, N, _ptr(u), _ptr(status), _stream(stream)))
    return u


def fine_solve_pcg(a: torch.Tensor, tol: float = 1e-12, max_iter: int = 500, u: torch.Tensor | None = None,
                   iters: torch.Tensor | None = None, status: torch.Tensor | None = None, stream=None):
    """Fine-grid FEM solutions by multigrid-preconditioned CG: returns
    (u[N][(nfine-1)^2], iters[N], status[N])."""
    assert a.dtype == torch.float64 and a.is_contiguous() and a.shape[1] == a.shape[2]
    N, nf = a.shape[0], a.shape[1]
    if u is None:
        u = torch.empty((N, (nf - 1) ** 2), dtype=torch.float64, device=a.device)
    if iters is None:
        iters = torch.empty(N, dtype=torch.int32, device=a.device)
    if status is None:
        status = torch.empty(N, dtype=torch.int32, device=a.device)
    _check("stomsfem_fine_solve_pcg", lib().stomsfem_fine_solve_pcg(
        _ptr(a), nf, N, tol, max_iter, _ptr(u), _ptr(iters), _ptr(status), _stream(stream)))
    return u, iters, status


def two_level_mc(U_H: torch.Tensor, U_Hh: torch.Tensor, u_fine: torch.Tensor, nc: int, m: int, stream=None):
    """Two-level MC estimate (mean, var_H, var_d) at the interior coarse nodes."""
    for t in (U_H, U_Hh, u_fine):
        assert t.dtype == torch.float64 and t.is_contiguous()
    assert U_Hh.shape[0] == u_fine.shape[0] and u_fine.shape[1] == (nc * m - 1) ** 2
    nU = (nc - 1) ** 2
    out = [torch.empty(nU, dtype=torch.float64, device=U_H.device) for _ in range(3)]
    _check("stomsfem_two_level_mc", lib().stomsfem_two_level_mc(
        _ptr(U_H), U_H.shape[0], _ptr(U_Hh), _ptr(u_fine), U_Hh.shape[0], nc, m, *[_ptr(t) for t in out],
        _stream(stream)))
    return tuple(out)


def upscale_os(a: torch.Tensor, ncx: int, ncy: int, m: int, oversample: int, S: torch.Tensor | None = None,
               status: torch.Tensor | None = None, stream=None):
    """Oversampled Petrov-Galerkin stiffness S[N][ncy*ncx][16] (row-major [trial][test])."""
    N = a.shape[0]
    if S is None:
        S = torch.empty((N, ncx * ncy, 16), dtype=torch.float64, device=a.device)
    assert S.is_contiguous()
    b = make_batch(a, ncx, ncy, m, S, status, entries=16)
    _check("stomsfem_upscale_os", lib().stomsfem_upscale_os(C.byref(b), oversample, _stream(stream)))
    return S


def coarse_solve_noalloc(S: torch.Tensor, ncx: int, ncy: int, U: torch.Tensor, qoi_mean: torch.Tensor | None = None,
                         qoi_var: torch.Tensor | None = None, status: torch.Tensor | None = None,
                         load: torch.Tensor | None = None, stream=None):
    """stomsfem_coarse_solve_noalloc: the coarse solve in the library's fixed
    device scratch (the library allocates nothing; outputs are the caller's)."""
    N = S.shape[0]
    assert S.dtype == torch.float64 and S.shape == (N, ncx * ncy, 10)
    assert U.dtype == torch.float64 and U.shape == (N, (ncx - 1) * (ncy - 1))
    _check("stomsfem_coarse_solve_noalloc", lib().stomsfem_coarse_solve_noalloc(
        ncx, ncy, N, _ptr(S), _ptr(load), _ptr(U), _ptr(qoi_mean), _ptr(qoi_var), _ptr(status), _stream(stream)))
    return U, qoi_mean, qoi_var


def coarse_solve_pg(S16: torch.Tensor, ncx: int, ncy: int, load: torch.Tensor | None = None,
                    U: torch.Tensor | None = None, qoi_mean: torch.Tensor | None = None,
                    qoi_var: torch.Tensor | None = None, status: torch.Tensor | None = None, stream=None):
    """Coarse solutions of the Petrov-Galerkin system from S16[N][ncy*ncx][16]."""
    N = S16.shape[0]
    assert S16.dtype == torch.float64 and S16.shape == (N, ncx * ncy, 16) and S16.is_contiguous()
    nU = (ncx - 1) * (ncy - 1)
    dev = S16.device
    if U is None:
        U = torch.empty((N, nU), dtype=torch.float64, device=dev)
    if qoi_mean is None:
        qoi_mean = torch.empty(nU, dtype=torch.float64, device=dev)
    if qoi_var is None:
        qoi_var = torch.empty(nU, dtype=torch.float64, device=dev)
    if load is not None:
        assert load.dtype == torch.float64 and load.shape == (ncx * ncy, 4)
    _check("stomsfem_coarse_solve_pg", lib().stomsfem_coarse_solve_pg(
        ncx, ncy, N, _ptr(S16), _ptr(load), _ptr(U), _ptr(qoi_mean), _ptr(qoi_var), _ptr(status), _stream(stream)))
    return U, qoi_mean, qoi_var


def workspace_reserve(nbytes: int):
    _check("stomsfem_workspace_reserve", lib().stomsfem_workspace_reserve(int(nbytes)))


def workspace_release():
    _check("stomsfem_workspace_release", lib().stomsfem_workspace_release())


class Model:
    """Owns a library model handle (freed with stomsfem_model_free)."""

    def __init__(self, handle, ncx, ncy, m):
        self.handle = handle
        self.ncx, self.ncy, self.m = ncx, ncy, m

    def free(self):
        if self.handle:
            lib().stomsfem_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def save(self, path: str):
        _check("stomsfem_model_save", lib().stomsfem_model_save(self.handle, os.fsencode(path)))

    def export(self, which: str):
        import numpy as np

        M = self.ncx * self.ncy
        nI = (getattr(self, "patch_m", self.m) - 1) ** 2
        spec = {"r": (0, np.int32, (M,)), "lambda": (1, np.float64, (M, nI)),
                "Z": (2, np.float64, (M, nI, 8)), "phibar": (3, np.float64, (M, 3, nI)),
                "offsets": (5, np.int64, (M + 1,))}
        if which == "table":
            rows = int(self.export("offsets")[-1])
            spec["table"] = (4, np.float64, (rows, 10))
        code, dt, shape = spec[which]
        out = np.zeros(shape, dtype=dt)
        _check("stomsfem_model_export", lib().stomsfem_model_export(
            self.handle, code, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out


def reduce(a_train: torch.Tensor, ncx: int, ncy: int, m: int, r_max: int = 8, tail_tol: float = 1e-6,
           stream=None) -> Model:
    """Offline reduced-basis build from training coefficients [Ntr][ncy*m][ncx*m]."""
    N = a_train.shape[0]
    assert a_train.shape[1:] == (ncy * m, ncx * m)
    b = Batch(ncx, ncy, m, _DT[a_train.dtype], N, _ptr(a_train), None, None)
    h = C.c_void_p()
    _check("stomsfem_reduce", lib().stomsfem_reduce(C.byref(b), r_max, tail_tol, C.byref(h), _stream(stream)))
    return Model(h, ncx, ncy, m)


def reduce_apply(model: Model, a: torch.Tensor, S: torch.Tensor | None = None,
                 status: torch.Tensor | None = None, precision: int = PREC_F32, stream=None):
    """Online reduced-basis upscaling S[N][M][10] for coefficient samples a."""
    N = a.shape[0]
    if S is None:
        S = torch.empty((N, model.ncx * model.ncy, 10), dtype=torch.float64, device=a.device)
    b = make_batch(a, model.ncx, model.ncy, model.m, S, status)
    _check("stomsfem_reduce_apply", lib().stomsfem_reduce_apply(model.handle, C.byref(b), precision,
                                                                _stream(stream)))
    return S


def reduce_os(a_train: torch.Tensor, ncx: int, ncy: int, m: int, oversample: int, r_max: int = 8,
              tail_tol: float = 1e-6, stream=None) -> Model:
    """Offline reduced-basis build on the oversampled patches (side m + 2 oversample)
    from training coefficients [Ntr][ncy*m][ncx*m]."""
    N = a_train.shape[0]
    assert a_train.shape[1:] == (ncy * m, ncx * m)
    b = Batch(ncx, ncy, m, _DT[a_train.dtype], N, _ptr(a_train), None, None)
    h = C.c_void_p()
    _check("stomsfem_reduce_os", lib().stomsfem_reduce_os(C.byref(b), oversample, r_max, tail_tol, C.byref(h),
                                                          _stream(stream)))
    md = Model(h, ncx, ncy, m)
    md.patch_m = m + 2 * oversample  # the exported patch quantities have (patch_m - 1)^2 interior nodes
    return md


def reduce_os_apply(model: Model, a: torch.Tensor, S: torch.Tensor | None = None,
                    status: torch.Tensor | None = None, precision: int = PREC_F64, stream=None):
    """Online Petrov-Galerkin stiffness S[N][M][16] from the reduced oversampled patches."""
    N = a.shape[0]
    if S is None:
        S = torch.empty((N, model.ncx * model.ncy, 16), dtype=torch.float64, device=a.device)
    b = make_batch(a, model.ncx, model.ncy, model.m, S, status, entries=16)
    _check("stomsfem_reduce_os_apply", lib().stomsfem_reduce_os_apply(model.handle, C.byref(b), precision,
                                                                      _stream(stream)))
    return S


def bump_family(wl) -> BumpFamily:
    p = wl.coef_params()
    return BumpFamily(p["g"], p["rho"], p["eps"], p["base"], p["amp"], p["beta"])


def local_vars_bumps(ncx: int, ncy: int, m: int, fam: BumpFamily, kmax: int = MLP_KIN):
    """Host computation of each patch's local variables -> (lv [M][kmax] int32, nlocal [M])."""
    import numpy as np

    M = ncx * ncy
    lv = np.zeros((M, kmax), dtype=np.int32)
    nl = np.zeros(M, dtype=np.int32)
    _check("stomsfem_local_vars_bumps", lib().stomsfem_local_vars_bumps(
        ncx, ncy, m, C.byref(fam), kmax, lv.ctypes.data_as(C.c_void_p), nl.ctypes.data_as(C.c_void_p)))
    return lv, nl


def mlp_create(ncx: int, ncy: int, m: int, lv, init_params, fam: BumpFamily, box: float = 1.0) -> Model:
    import numpy as np

    lv = np.ascontiguousarray(lv, dtype=np.int32)
    ip = np.ascontiguousarray(init_params, dtype=np.float32)
    assert ip.shape == (ncx * ncy, MLP_NPARAM) and lv.shape == (ncx * ncy, MLP_KIN)
    h = C.c_void_p()
    _check("stomsfem_mlp_create", lib().stomsfem_mlp_create(
        ncx, ncy, m, lv.ctypes.data_as(C.c_void_p), ip.ctypes.data_as(C.c_void_p), C.byref(fam), box, C.byref(h)))
    return Model(h, ncx, ncy, m)


def local_vars_features(ncx: int, ncy: int, m: int, fmap, nfeat: int, kmax: int = MLP_KIN):
    """Host computation of each patch's features from a host map -> (lv [M][kmax] int32, nlocal [M])."""
    import numpy as np

    fm = np.ascontiguousarray(fmap, dtype=np.int32)
    assert fm.shape == (ncy * m, ncx * m)
    M = ncx * ncy
    lv = np.zeros((M, kmax), dtype=np.int32)
    nl = np.zeros(M, dtype=np.int32)
    _check("stomsfem_local_vars_features", lib().stomsfem_local_vars_features(
        ncx, ncy, m, fm.ctypes.data_as(C.c_void_p), nfeat, kmax, lv.ctypes.data_as(C.c_void_p),
        nl.ctypes.data_as(C.c_void_p)))
    return lv, nl


def mlp_create_features(nc: int, m: int, fmap: torch.Tensor, nfeat: int, decades: float, init_params,
                        box: float = 1.0) -> Model:
    """Surrogate of the channels medium; fmap device int32 [nc*m][nc*m]."""
    import numpy as np

    assert fmap.dtype == torch.int32 and fmap.is_contiguous() and tuple(fmap.shape) == (nc * m, nc * m)
    ip = np.ascontiguousarray(init_params, dtype=np.float32)
    assert ip.shape == (nc * nc, MLP_NPARAM)
    h = C.c_void_p()
    _check("stomsfem_mlp_create_features", lib().stomsfem_mlp_create_features(
        nc, m, _ptr(fmap), nfeat, decades, ip.ctypes.data_as(C.c_void_p), box, C.byref(h)))
    return Model(h, nc, nc, m)


def mlp_set_data(model: Model, xi: torch.Tensor, S: torch.Tensor, stream=None):
    assert xi.dtype == torch.float64 and S.dtype == torch.float64
    _check("stomsfem_mlp_set_data", lib().stomsfem_mlp_set_data(
        model.handle, _ptr(xi), xi.shape[1], _ptr(S), xi.shape[0], _stream(stream)))


def mlp_train(model: Model, steps: int, lr: float, perm: torch.Tensor | None = None, loss: torch.Tensor | None = None,
              stream=None):
    _check("stomsfem_mlp_train", lib().stomsfem_mlp_train(model.handle, steps, lr, _ptr(perm), _ptr(loss),
                                                          _stream(stream)))


def mlp_grad(model: Model, xb: torch.Tensor, tb: torch.Tensor, stream=None):
    M = model.ncx * model.ncy
    grads = torch.empty((M, MLP_NPARAM), dtype=torch.float32, device=xb.device)
    loss = torch.empty(M, dtype=torch.float32, device=xb.device)
    _check("stomsfem_mlp_grad", lib().stomsfem_mlp_grad(model.handle, _ptr(xb), _ptr(tb), _ptr(grads), _ptr(loss),
                                                        _stream(stream)))
    return grads, loss


def mlp_params(model: Model, stream=None) -> torch.Tensor:
    out = torch.empty((model.ncx * model.ncy, MLP_NPARAM), dtype=torch.float32, device="cuda")
    _check("stomsfem_mlp_params", lib().stomsfem_mlp_params(model.handle, _ptr(out), None, _stream(stream)))
    return out


def mlp_standardization(model: Model):
    import numpy as np

    M = model.ncx * model.ncy
    mu = np.zeros((M, 10))
    sd = np.zeros((M, 10))
    _check("stomsfem_mlp_standardization", lib().stomsfem_mlp_standardization(
        model.handle, mu.ctypes.data_as(C.c_void_p), sd.ctypes.data_as(C.c_void_p)))
    return mu, sd


def mlp_predict(model: Model, xi: torch.Tensor, precision: int = PREC_BF16, stream=None) -> torch.Tensor:
    N = xi.shape[0]
    Y = torch.empty((N, model.ncx * model.ncy, 20), dtype=torch.float32, device=xi.device)
    _check("stomsfem_mlp_predict", lib().stomsfem_mlp_predict(model.handle, _ptr(xi), xi.shape[1], N, _ptr(Y),
                                                              precision, _stream(stream)))
    return Y


def mlp_gate(model: Model, Y: torch.Tensor, xi: torch.Tensor, gate_tol: float = 1e-3, stream=None):
    """The surrogate's gate on given raw outputs Y[N][M][20]: returns
    (S[N][M][10], status[N][M] (0 accepted, 1 rejected), gate[N][M][2])."""
    N = xi.shape[0]
    M = model.ncx * model.ncy
    S = torch.empty((N, M, 10), dtype=torch.float64, device=xi.device)
    status = torch.empty((N, M), dtype=torch.int32, device=xi.device)
    gate = torch.empty((N, M, 2), dtype=torch.float64, device=xi.device)
    _check("stomsfem_mlp_gate", lib().stomsfem_mlp_gate(model.handle, _ptr(Y), _ptr(xi), xi.shape[1], N, gate_tol,
                                                        _ptr(S), _ptr(status), _ptr(gate), _stream(stream)))
    return S, status, gate


def upscale_surrogate(model: Model, xi: torch.Tensor, gate_tol: float = 1e-3, precision: int = PREC_BF16,
                      S: torch.Tensor | None = None, status: torch.Tensor | None = None,
                      stats: torch.Tensor | None = None, stream=None):
    N = xi.shape[0]
    M = model.ncx * model.ncy
    if S is None:
        S = torch.empty((N, M, 10), dtype=torch.float64, device=xi.device)
    _check("stomsfem_upscale_surrogate", lib().stomsfem_upscale_surrogate(
        model.handle, _ptr(xi), xi.shape[1], N, _ptr(S), _ptr(status), gate_tol, precision, _ptr(stats),
        _stream(stream)))
    return S


def interp_build(ncx: int, ncy: int, m: int, lv, fam: BumpFamily, nnodes: int, lo: float = -1.0, hi: float = 1.0,
                 stream=None) -> Model:
    """Offline random interpolation: S at the tensor Chebyshev-Gauss-Lobatto
    nodes of every patch's local variables (lv [M][4], -1 padded)."""
    import numpy as np

    lv = np.ascontiguousarray(lv, dtype=np.int32)
    assert lv.shape == (ncx * ncy, MLP_KIN)
    h = C.c_void_p()
    _check("stomsfem_interp_build", lib().stomsfem_interp_build(
        ncx, ncy, m, lv.ctypes.data_as(C.c_void_p), C.byref(fam), nnodes, lo, hi, C.byref(h), _stream(stream)))
    return Model(h, ncx, ncy, m)


def interp_apply(model: Model, xi: torch.Tensor, S: torch.Tensor | None = None, status: torch.Tensor | None = None,
                 stream=None):
    """Online random interpolation S[N][M][10]; returns (S, number of pairs
    computed by the plain path because a local variable left the box)."""
    assert xi.dtype == torch.float64
    N = xi.shape[0]
    if S is None:
        S = torch.empty((N, model.ncx * model.ncy, 10), dtype=torch.float64, device=xi.device)
    nfb = C.c_int64(0)
    _check("stomsfem_interp_apply", lib().stomsfem_interp_apply(
        model.handle, _ptr(xi), xi.shape[1], N, _ptr(S), _ptr(status), C.byref(nfb), _stream(stream)))
    return S, nfb.value


def sparse_grid(dim: int, level: int):
    """Smolyak Clenshaw-Curtis grid (host): (digits int32 [n][dim], weights [n])."""
    import numpy as np

    n = C.c_int64(0)
    _check("stomsfem_sparse_grid", lib().stomsfem_sparse_grid(dim, level, 0, C.byref(n), None, None))
    dg = np.zeros((n.value, dim), dtype=np.int32)
    w = np.zeros(n.value, dtype=np.float64)
    _check("stomsfem_sparse_grid", lib().stomsfem_sparse_grid(
        dim, level, n.value, C.byref(n), dg.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p)))
    return dg, w


def sc_build(ncx: int, ncy: int, m: int, lv, fam: BumpFamily, level: int, digits, lo: float = -1.0,
             hi: float = 1.0, stream=None) -> Model:
    """Offline dictionaries of S at the distinct local collocation points of
    every patch for the collocation points `digits` (host int32 [n][g*g])."""
    import numpy as np

    lv = np.ascontiguousarray(lv, dtype=np.int32)
    assert lv.shape == (ncx * ncy, MLP_KIN)
    dg = np.ascontiguousarray(digits, dtype=np.int32)
    h = C.c_void_p()
    _check("stomsfem_sc_build", lib().stomsfem_sc_build(
        ncx, ncy, m, lv.ctypes.data_as(C.c_void_p), C.byref(fam), level, lo, hi, dg.ctypes.data_as(C.c_void_p),
        dg.shape[0], C.byref(h), _stream(stream)))
    return Model(h, ncx, ncy, m)


def sc_apply(model: Model, digits: torch.Tensor, S: torch.Tensor | None = None, status: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
    """Online search and plug-in: S [n][M][10] for digits (device int32 [n][nxi])."""
    assert digits.dtype == torch.int32 and digits.is_contiguous()
    n = digits.shape[0]
    if S is None:
        S = torch.empty((n, model.ncx * model.ncy, 10), dtype=torch.float64, device=digits.device)
    _check("stomsfem_sc_apply", lib().stomsfem_sc_apply(
        model.handle, _ptr(digits), digits.shape[1], n, _ptr(S), _ptr(status), _stream(stream)))
    return S


def sgi_build(ncx: int, ncy: int, m: int, lv, fam: BumpFamily, level: int, lo: float = -1.0, hi: float = 1.0,
              stream=None) -> Model:
    """Offline sparse-grid interpolation: S at the level-`level` Smolyak
    Clenshaw-Curtis nodes of every patch's local variables."""
    import numpy as np

    lv = np.ascontiguousarray(lv, dtype=np.int32)
    assert lv.shape == (ncx * ncy, MLP_KIN)
    h = C.c_void_p()
    _check("stomsfem_sgi_build", lib().stomsfem_sgi_build(
        ncx, ncy, m, lv.ctypes.data_as(C.c_void_p), C.byref(fam), level, lo, hi, C.byref(h), _stream(stream)))
    return Model(h, ncx, ncy, m)


def sgi_apply(model: Model, xi: torch.Tensor, S: torch.Tensor | None = None, status: torch.Tensor | None = None,
              stream=None):
    """Online sparse-grid interpolation S[N][M][10]; returns (S, number of
    pairs computed by the plain path because a local variable left the box)."""
    assert xi.dtype == torch.float64
    N = xi.shape[0]
    if S is None:
        S = torch.empty((N, model.ncx * model.ncy, 10), dtype=torch.float64, device=xi.device)
    nfb = C.c_int64(0)
    _check("stomsfem_sgi_apply", lib().stomsfem_sgi_apply(
        model.handle, _ptr(xi), xi.shape[1], N, _ptr(S), _ptr(status), C.byref(nfb), _stream(stream)))
    return S, nfb.value


def quadrature(U: torch.Tensor, w: torch.Tensor, mean: torch.Tensor | None = None, var: torch.Tensor | None = None,
               stream=None):
    """Collocation estimates (sum_p w_p U_p, sum_p w_p U_p^2 - mean^2)."""
    assert U.dtype == torch.float64 and w.dtype == torch.float64 and U.is_contiguous()
    n, nu = U.shape
    if mean is None:
        mean = torch.empty(nu, dtype=torch.float64, device=U.device)
    if var is None:
        var = torch.empty(nu, dtype=torch.float64, device=U.device)
    _check("stomsfem_quadrature", lib().stomsfem_quadrature(_ptr(U), _ptr(w), n, nu, _ptr(mean), _ptr(var),
                                                           _stream(stream)))
    return mean, var


def feature_map(nfine: int, kind: torch.Tensor, x0: torch.Tensor, y0: torch.Tensor, size: torch.Tensor,
                stream=None) -> torch.Tensor:
    """Index of the highest feature covering each fine element (-1: background)."""
    out = torch.empty((nfine, nfine), dtype=torch.int32, device=kind.device)
    _check("stomsfem_feature_map", lib().stomsfem_feature_map(
        nfine, kind.shape[0], _ptr(kind), _ptr(x0), _ptr(y0), _ptr(size), _ptr(out), _stream(stream)))
    return out


def coef_features(fmap: torch.Tensor, nfeat: int, xi: torch.Tensor, decades: float = 4.0, dtype=torch.float64,
                  out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Coefficient samples a[N][nfine][nfine] of the channels-and-inclusions medium."""
    assert xi.dtype == torch.float64 and fmap.dtype == torch.int32
    N, nxi = xi.shape
    nfine = fmap.shape[0]
    if out is None:
        out = torch.empty((N, nfine, nfine), dtype=dtype, device=xi.device)
    _check("stomsfem_coef_features", lib().stomsfem_coef_features(
        N, nfine, _ptr(fmap), nfeat, _ptr(xi), nxi, decades, _ptr(out), _DT[out.dtype], _stream(stream)))
    return out


FAMILY_BUMPS, FAMILY_FEATURES = 0, 1


def make_stage(nc: int, m: int, xi: torch.Tensor, *, bumps: BumpFamily | None = None,
               feature_map: torch.Tensor | None = None, nfeat: int = 0, decades: float = 4.0,
               a_dtype=torch.float64, U: torch.Tensor | None = None, qoi_mean: torch.Tensor | None = None,
               qoi_var: torch.Tensor | None = None, status: torch.Tensor | None = None) -> Stage:
    """Descriptor of one plan stage (the tensors must outlive the plan)."""
    assert xi.dtype == torch.float64 and xi.is_contiguous()
    fam = bumps if bumps is not None else BumpFamily(0, 0.0, 0.0, 0.0, 0.0, 0.0)
    return Stage(nc, nc, m, xi.shape[0], _DT[a_dtype], FAMILY_BUMPS if bumps is not None else FAMILY_FEATURES, fam,
                 _ptr(feature_map), nfeat, decades, _ptr(xi), xi.shape[1], _ptr(U), _ptr(qoi_mean), _ptr(qoi_var),
                 _ptr(status))


class Plan:
    """Owns a library execution plan (stomsfem_plan_free on release)."""

    def __init__(self, handle, nstage):
        self.handle = handle
        self.nstage = nstage

    def launch(self, stage: int = -1, stream=None):
        _check("stomsfem_plan_launch", lib().stomsfem_plan_launch(self.handle, stage, _stream(stream)))

    def free(self):
        if self.handle:
            lib().stomsfem_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def plan_create(stages: list[Stage]) -> Plan:
    arr = (Stage * len(stages))(*stages)
    h = C.c_void_p()
    _check("stomsfem_plan_create", lib().stomsfem_plan_create(arr, len(stages), C.byref(h)))
    return Plan(h, len(stages))


def autotune(a: torch.Tensor, ncx: int, ncy: int, m: int, S: torch.Tensor | None = None, reps: int = 5,
             stream=None) -> dict:
    """Tune the plain upscaling kernels for this batch's (m, dtype); the choice
    is used by later calls in this process.  Returns the tuner's report."""
    N = a.shape[0]
    if S is None:
        S = torch.empty((N, ncx * ncy, 10), dtype=torch.float64, device=a.device)
    b = make_batch(a, ncx, ncy, m, S, None)
    t = Tuning()
    _check("stomsfem_autotune", lib().stomsfem_autotune(C.byref(b), reps, C.byref(t), _stream(stream)))
    return {f: getattr(t, f) for f, _ in Tuning._fields_}


def tuning_reset():
    _check("stomsfem_tuning_reset", lib().stomsfem_tuning_reset())


def model_load(path: str) -> Model:
    """Load a model file written by Model.save onto the current device."""
    h = C.c_void_p()
    _check("stomsfem_model_load", lib().stomsfem_model_load(os.fsencode(path), C.byref(h)))
    kind, ncx, ncy, m = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check("stomsfem_model_shape", lib().stomsfem_model_shape(h, C.byref(kind), C.byref(ncx), C.byref(ncy),
                                                             C.byref(m)))
    return Model(h, ncx.value, ncy.value, m.value)


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("refine_pairs", "refine_recomputed", "interp_pairs", "interp_fallbacks",
                                          "surrogate_pairs", "surrogate_recomputed")]


def stats_get() -> dict:
    st = Stats()
    _check("stomsfem_stats_get", lib().stomsfem_stats_get(C.byref(st)))
    return {f: getattr(st, f) for f, _ in Stats._fields_}


def stats_reset():
    _check("stomsfem_stats_reset", lib().stomsfem_stats_reset())
