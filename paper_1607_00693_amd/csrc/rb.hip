// Reduced-basis upscaling (Sec. 3.2, eqs. KLphi, localRB, localRBsystem,
// RBaffine / localAF; Algorithms 3 and 4).
//
// Offline (per patch K, from N_train coefficient samples):
//   cell_phi_kernel  -- the cell-problem solutions phi^l(xi_s), l = 0..2, on
//                       the interior nodes (banded LDL^T in LDS, one
//                       wavefront per pair, forward and backward solves);
//                       where that band does not fit LDS the refined
//                       FP32/FP64 kernel of upscale_mixed.hip supplies them;
//   rb_build_kernel  -- primal form (3 N_train >= nI), one workgroup per
//                       patch: mean phibar^l, centred snapshot Gram
//                       H = Psi Psi^T, energy matrix E = K_II(abar) =
//                       L_E L_E^T with abar the training mean of the
//                       coefficient, C = L_E^T H L_E (the Gram matrix of the
//                       KL expansion in the energy inner product), cyclic
//                       Jacobi eigen-decomposition C = V Lambda V^T, the tail
//                       rule for r, modes Z = L_E^{-T} V_r (Z^T E Z = I), and
//                       the element table G;
//   rb_dual_*        -- dual form (3 N_train < nI, the method of snapshots):
//                       W = E Psi, the ns x ns Gram C = Psi^T W in tiles,
//                       its eigenpairs, modes z_q = Psi v_q / sqrt(lambda_q)
//                       (the same KL subspace and eigenvalues), the table G.
// The Q1 stiffness is affine in the per-element coefficient values
// (K(a) = sum_e a_e K_e), which is the paper's affine structure taken at
// element level: every quantity of the online Galerkin system is a linear
// function of the patch's m*m coefficient values,
//     A_qq'  = sum_e a_e zeta_q . K_e zeta_q'           (r(r+1)/2 values)
//     Fh_lq  = sum_e a_e zeta_q . K_e phibar^l          (3 r values)
//     B_ll'  = sum_e a_e phibar^l . K_e phibar^l'       (6 values)
// (phibar^l carries the Dirichlet data g^l on the boundary).  G holds these
// P per-element coefficients, so the online stage is one GEMM
// [pairs x m*m] x [m*m x P] per patch, then an r x r Cholesky per pair and
//     S_ll' = B_ll' - Fh_l . A^{-1} Fh_l'
// (Galerkin identity: phi_rb = phibar + Z c with A c = -Fh).
//
// Online: rb_apply_mfma_kernel (FP32 MFMA 16x16x4, FP32 accumulation, FP32
// r x r solve) and rb_apply_f64_kernel (FP64 throughout, for parity checks).
#include "rb.h"
#include "rb_os_dev.h"

#include <type_traits>

namespace stomsfem {

// ---------------------------------------------------------------------------
// Cell-problem solutions (snapshots)
// ---------------------------------------------------------------------------
struct PhiArgs {
  UpArgs up;
  double* phi;  // [npairs][3][nI]
};

template <typename TA>
__global__ __launch_bounds__(64) void cell_phi_kernel(PhiArgs pa) {
  extern __shared__ double smem[];
  const UpArgs& args = pa.up;
  const int m = args.m, n = m - 1, nI = n * n, B = m;
  double* A = smem;            // m*m
  double* Bd = A + m * m;      // nI*(B+1): Bd[i*(B+1)+d] = K(i, i-d), column j kept unscaled
  double* F = Bd + nI * (B + 1);  // 3*nI
  const int tid = threadIdx.x;
  const int Mc = args.ncx * args.ncy;
  const int64_t lda = (int64_t)args.ncx * m;
  for (int64_t p = blockIdx.x; p < args.npairs; p += gridDim.x) {
    const int64_t s = p / Mc;
    const int K = (int)(p - s * Mc);
    const TA* a = (const TA*)args.a + block_offset(s, K, args.ncx, args.ncy, m);
    __syncthreads();
    for (int i = tid; i < m * m; i += blockDim.x) A[i] = ld(a, (i / m) * lda + (i % m));
    __syncthreads();
    for (int r = tid; r < nI; r += blockDim.x) {
      const int ix = r % n, iy = r / n, px = ix + 1, py = iy + 1;
      const double aSW = A[iy * m + ix], aSE = A[iy * m + ix + 1];
      const double aNW = A[(iy + 1) * m + ix], aNE = A[(iy + 1) * m + ix + 1];
      double* row = Bd + r * (B + 1);
      for (int d = 0; d <= B; ++d) row[d] = 0.0;
      row[0] = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
      const int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
      const int dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
      const double ks[8] = {-(aSW + aNW) / 6.0, -(aSE + aNE) / 6.0, -(aSW + aSE) / 6.0, -(aNW + aNE) / 6.0,
                            -aSW / 3.0,         -aSE / 3.0,         -aNW / 3.0,         -aNE / 3.0};
      double f[3] = {0, 0, 0};
      for (int q = 0; q < 8; ++q) {
        const int qx = px + dxs[q], qy = py + dys[q];
        if (qx == 0 || qx == m || qy == 0 || qy == m) {
          for (int l = 0; l < 3; ++l) f[l] -= ks[q] * pcorner(l, qx, qy, m);
        } else {
          const int c = (qy - 1) * n + (qx - 1);
          if (c < r) row[r - c] = ks[q];
        }
      }
      for (int l = 0; l < 3; ++l) F[l * nI + r] = f[l];
    }
    __syncthreads();
    // right-looking LDL^T, column j kept unscaled (W_ij = l_ij d_j)
    for (int j = 0; j < nI; ++j) {
      const double d = Bd[j * (B + 1)];
      const double inv = 1.0 / d;
      const int cnt = (j + B < nI - 1 ? j + B : nI - 1) - j;
      const int npairs = cnt * (cnt + 1) / 2;
      for (int q = tid; q < npairs; q += blockDim.x) {
        int io = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
        while (io * (io + 1) / 2 > q) --io;
        while ((io + 1) * (io + 2) / 2 <= q) ++io;
        const int ko = q - io * (io + 1) / 2;
        const int i = j + 1 + io, k = j + 1 + ko;
        Bd[i * (B + 1) + (i - k)] -= Bd[i * (B + 1) + (i - j)] * inv * Bd[k * (B + 1) + (k - j)];
      }
      for (int t = tid; t < 3 * cnt; t += blockDim.x) {
        const int i = j + 1 + t / 3, l = t % 3;
        F[l * nI + i] -= Bd[i * (B + 1) + (i - j)] * inv * F[l * nI + j];
      }
      __syncthreads();
    }
    // backward: x_j = (y_j - sum_{t=1..B} W_{j+t,j} x_{j+t}) / d_j
    if (tid < 3) {
      double* x = F + tid * nI;
      for (int j = nI - 1; j >= 0; --j) {
        double v = x[j];
        const int t1 = (j + B < nI - 1 ? j + B : nI - 1) - j;
        for (int t = 1; t <= t1; ++t) v -= Bd[(j + t) * (B + 1) + t] * x[j + t];
        x[j] = v / Bd[j * (B + 1)];
      }
    }
    __syncthreads();
    for (int i = tid; i < 3 * nI; i += blockDim.x) pa.phi[p * 3 * nI + i] = F[i];
  }
}

size_t cell_phi_lds_bytes(int m) {
  const int nI = (m - 1) * (m - 1);
  return sizeof(double) * ((size_t)m * m + (size_t)nI * (m + 1) + 3 * (size_t)nI);
}

hipError_t launch_cell_phi(const UpArgs& args, int a_dtype, double* phi, hipStream_t st) {
  PhiArgs pa{args, phi};
  const int64_t blocks = args.npairs < 65536 ? args.npairs : 65536;
  if (blocks == 0) return hipSuccess;
  const size_t lds = cell_phi_lds_bytes(args.m);
  if (lds > CELL_PHI_LDS_MAX) return hipErrorInvalidValue;
  // above 64 KB the kernel's dynamic-LDS limit is raised on the current
  // device before the launch
  hipError_t e = hipSuccess;
  if (a_dtype == STOMSFEM_F32) {
    if (lds > 65536)
      e = hipFuncSetAttribute((const void*)cell_phi_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e == hipSuccess) hipLaunchKernelGGL(cell_phi_kernel<float>, dim3((unsigned)blocks), dim3(64), lds, st, pa);
  } else {
    if (lds > 65536)
      e = hipFuncSetAttribute((const void*)cell_phi_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e == hipSuccess) hipLaunchKernelGGL(cell_phi_kernel<double>, dim3((unsigned)blocks), dim3(64), lds, st, pa);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

// Snapshots of cells whose band does not fit a workgroup's LDS (used for
// m > 32, past the refined kernel).  One wavefront per pair.  The band rows
// j .. j+B of the elimination window sit in a circular LDS ring of B+1 rows
// (row i in slot i mod (B+1), entry d = K(i, i-d), column j kept unscaled as
// in cell_phi_kernel); the three lifts are forward-substituted in the same
// pivot loop.  A row leaves the ring after its pivot, finished, to the
// workgroup's global row store with its forward-substituted right-hand
// sides, and the backward substitution reads the stored rows in reverse: the
// B products of a step are taken by the lanes and reduced over the
// wavefront, the next step's entries fetched one step ahead.
struct PhiBandArgs {
  UpArgs up;
  double* phi;   // [npairs][3][nI]
  double* rows;  // [gridDim.x][nI][B+1] finished rows
  double* ys;    // [gridDim.x][3][nI] forward-substituted right-hand sides
};

#define RB_WAVE_SYNC()                                     \
  do {                                                     \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                       \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
  } while (0)

template <typename TA>
__global__ __launch_bounds__(64) void cell_phi_band_kernel(PhiBandArgs pa) {
  extern __shared__ double smem[];
  const UpArgs& args = pa.up;
  const int m = args.m, n = m - 1, nI = n * n, B = m, W = B + 1;
  double* Wn = smem;          // [W][W] ring of band rows
  double* Fr = Wn + W * W;    // [3][W] right-hand sides of the ring rows
  double* Xr = Fr + 3 * W;    // [3][W] solution values of the last B rows (backward pass)
  const int lane = threadIdx.x;
  const int Mc = args.ncx * args.ncy;
  const int64_t lda = (int64_t)args.ncx * m;
  double* rows = pa.rows + (int64_t)blockIdx.x * nI * W;
  double* ys = pa.ys + (int64_t)blockIdx.x * 3 * nI;
  for (int64_t p = blockIdx.x; p < args.npairs; p += gridDim.x) {
    const int64_t s = p / Mc;
    const int K = (int)(p - s * Mc);
    const TA* a = (const TA*)args.a + block_offset(s, K, args.ncx, args.ncy, m);
    // row r of K_II into slot r mod W and its lifts (the stencil of cell_phi_kernel)
    auto build = [&](int r) {
      double* row = Wn + (r % W) * W;
      for (int d = lane; d <= B; d += 64) row[d] = 0.0;
      RB_WAVE_SYNC();
      if (lane == 0) {
        const int ix = r % n, iy = r / n, px = ix + 1, py = iy + 1;
        const double aSW = ld(a, (int64_t)iy * lda + ix), aSE = ld(a, (int64_t)iy * lda + ix + 1);
        const double aNW = ld(a, (int64_t)(iy + 1) * lda + ix), aNE = ld(a, (int64_t)(iy + 1) * lda + ix + 1);
        row[0] = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
        const int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
        const int dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
        const double ks[8] = {-(aSW + aNW) / 6.0, -(aSE + aNE) / 6.0, -(aSW + aSE) / 6.0, -(aNW + aNE) / 6.0,
                              -aSW / 3.0,         -aSE / 3.0,         -aNW / 3.0,         -aNE / 3.0};
        double f[3] = {0, 0, 0};
        for (int q = 0; q < 8; ++q) {
          const int qx = px + dxs[q], qy = py + dys[q];
          if (qx == 0 || qx == m || qy == 0 || qy == m) {
            for (int l = 0; l < 3; ++l) f[l] -= ks[q] * pcorner(l, qx, qy, m);
          } else {
            const int c = (qy - 1) * n + (qx - 1);
            if (c < r) row[r - c] = ks[q];
          }
        }
        for (int l = 0; l < 3; ++l) Fr[l * W + r % W] = f[l];
      }
      RB_WAVE_SYNC();
    };
    for (int r = 0; r < W && r < nI; ++r) build(r);
    for (int j = 0; j < nI; ++j) {
      const int sj = j % W;
      const double inv = 1.0 / Wn[sj * W];
      const int cnt = (j + B < nI - 1 ? j + B : nI - 1) - j;
      const int npr = cnt * (cnt + 1) / 2;
      for (int q = lane; q < npr; q += 64) {
        int io = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
        while (io * (io + 1) / 2 > q) --io;
        while ((io + 1) * (io + 2) / 2 <= q) ++io;
        const int ko = q - io * (io + 1) / 2;
        const int i = j + 1 + io, k = j + 1 + ko;
        Wn[(i % W) * W + (i - k)] -= Wn[(i % W) * W + (i - j)] * inv * Wn[(k % W) * W + (k - j)];
      }
      for (int t = lane; t < 3 * cnt; t += 64) {
        const int i = j + 1 + t / 3, l = t % 3;
        Fr[l * W + i % W] -= Wn[(i % W) * W + (i - j)] * inv * Fr[l * W + sj];
      }
      RB_WAVE_SYNC();
      // row j is finished: to the row store, its slot to the row entering at j + W
      for (int d = lane; d <= B; d += 64) rows[(int64_t)j * W + d] = Wn[sj * W + d];
      if (lane < 3) ys[(int64_t)lane * nI + j] = Fr[lane * W + sj];
      RB_WAVE_SYNC();
      if (j + W < nI) build(j + W);
    }
    // the stored rows are read back by other lanes of the wavefront
    __threadfence();
    __syncthreads();
    // backward: x_j = (y_j - sum_{t=1..B} W_{j+t,j} x_{j+t}) / d_j; lane t
    // takes t (lane 0 takes t = 64 when B = 64)
    const int t = lane == 0 ? 64 : lane;
    const bool tl = t <= B;
    auto fetch = [&](int j) { return (j >= 0 && tl && j + t < nI) ? rows[(int64_t)(j + t) * W + t] : 0.0; };
    double wc = fetch(nI - 1);
    double* out = pa.phi + p * 3 * nI;
    for (int j = nI - 1; j >= 0; --j) {
      const double wn = fetch(j - 1);
      double v[3];
      const bool on = tl && j + t < nI;
#pragma unroll
      for (int l = 0; l < 3; ++l) v[l] = on ? wc * Xr[l * W + (j + t) % W] : 0.0;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int l = 0; l < 3; ++l) v[l] += __shfl_xor(v[l], off, 64);
      if (lane < 3) {
        const double x = (ys[(int64_t)lane * nI + j] - v[lane]) / rows[(int64_t)j * W];
        Xr[lane * W + j % W] = x;
        out[(int64_t)lane * nI + j] = x;
      }
      RB_WAVE_SYNC();
      wc = wn;
    }
    __syncthreads();  // the ring and the row store are reused by the next pair
  }
}

size_t cell_phi_band_lds_bytes(int m) {
  const size_t W = (size_t)m + 1;
  return sizeof(double) * (W * W + 6 * W);
}

int64_t cell_phi_band_ws_doubles(int m) {
  const int64_t nI = (int64_t)(m - 1) * (m - 1);
  return nI * (m + 1) + 3 * nI;
}

hipError_t launch_cell_phi_band(const UpArgs& args, int a_dtype, double* phi, double* ws, int64_t blocks,
                                hipStream_t st) {
  if (args.npairs == 0) return hipSuccess;
  if (args.m < 2 || args.m > 64 || blocks < 1) return hipErrorInvalidValue;
  const int64_t nI = (int64_t)(args.m - 1) * (args.m - 1);
  if (blocks > args.npairs) blocks = args.npairs;
  PhiBandArgs pa{args, phi, ws, ws + blocks * nI * (args.m + 1)};
  const size_t lds = cell_phi_band_lds_bytes(args.m);
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(cell_phi_band_kernel<float>, dim3((unsigned)blocks), dim3(64), lds, st, pa);
  else
    hipLaunchKernelGGL(cell_phi_band_kernel<double>, dim3((unsigned)blocks), dim3(64), lds, st, pa);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Offline build
// ---------------------------------------------------------------------------
constexpr int RB_THREADS = 256;
constexpr int RB_NMAX = 1024;  // largest eigenproblem (primal nI or dual 3 ntrain)

// Cyclic Jacobi on the symmetric n x n matrix H (global, overwritten by its
// rotated form, whose diagonal ends up holding the eigenvalues); V receives
// the eigenvectors as columns.  Rotations in the (p, q) planes (Golub and
// Van Loan's symmetric Schur pair) until the off-diagonal mass is below
// 1e-30 of the diagonal's.  Whole workgroup.
__device__ void rb_jacobi(double* H, double* V, int n, int max_sweeps, double* red, double* rot) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int ij = tid; ij < n * n; ij += nt) V[ij] = (ij / n == ij % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int ij = tid; ij < n * n; ij += nt) {  // symmetrise (rounding)
    const int i = ij / n, j = ij % n;
    if (j > i) {
      const double v = 0.5 * (H[i * n + j] + H[j * n + i]);
      H[i * n + j] = v;
      H[j * n + i] = v;
    }
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int ij = tid; ij < n * n; ij += nt) {
      const double v = H[ij] * H[ij];
      if (ij / n == ij % n) dia += v; else off += v;
    }
    red[tid] = off;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = dia;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double dias = red[0];
    __syncthreads();
    if (!(offs > 1e-30 * dias)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (tid == 0) {
          const double apq = H[p * n + q];
          double c = 1.0, s = 0.0;
          if (apq != 0.0) {
            const double tau = (H[q * n + q] - H[p * n + p]) / (2.0 * apq);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
          rot[0] = c;
          rot[1] = s;
        }
        __syncthreads();
        const double c = rot[0], s = rot[1];
        if (s != 0.0) {
          for (int k = tid; k < n; k += nt) {
            const double hp = H[k * n + p], hq = H[k * n + q];
            H[k * n + p] = c * hp - s * hq;
            H[k * n + q] = s * hp + c * hq;
            const double vp = V[k * n + p], vq = V[k * n + q];
            V[k * n + p] = c * vp - s * vq;
            V[k * n + q] = s * vp + c * vq;
          }
          __syncthreads();
          for (int k = tid; k < n; k += nt) {
            const double hp = H[p * n + k], hq = H[q * n + k];
            H[p * n + k] = c * hp - s * hq;
            H[q * n + k] = s * hp + c * hq;
          }
        }
        __syncthreads();
      }
  }
}

// Eigenvalues (the diagonal of the rotated H) in descending order into
// order[] / lambda[0..nlam) (zeros beyond n), and the number of modes:
// r = min(rcap, rmax, n, smallest r whose relative tail
// sqrt(sum_{q>r} lambda_q / sum lambda_q) <= tail_tol, number of eigenvalues
// above RB_RANK_TOL lambda_max).  Thread 0; the caller synchronises.
constexpr double RB_RANK_TOL = 1e-12;
__device__ int rb_sort_tail(const double* H, int n, int* order, double tail_tol, int rcap, int rmax, double* lambda,
                            int nlam) {
  for (int i = 0; i < n; ++i) order[i] = i;
  for (int i = 0; i < n; ++i) {  // selection sort
    int best = i;
    for (int j = i + 1; j < n; ++j)
      if (H[order[j] * n + order[j]] > H[order[best] * n + order[best]]) best = j;
    const int t = order[i];
    order[i] = order[best];
    order[best] = t;
  }
  double tot = 0.0;
  for (int i = 0; i < n; ++i) tot += fmax(H[order[i] * n + order[i]], 0.0);
  int r = n;
  double tail = tot;
  for (int q = 1; q <= n; ++q) {
    tail -= fmax(H[order[q - 1] * n + order[q - 1]], 0.0);
    const double rel = tot > 0 ? sqrt(fmax(tail, 0.0) / tot) : 0.0;
    if (rel <= tail_tol) {
      r = q;
      break;
    }
  }
  if (r > rcap) r = rcap;
  if (r > rmax) r = rmax;
  if (r > n) r = n;
  // numerical rank of the snapshots: eigenvalues at or below 1e-12 of the
  // largest are rounding, not modes (the method of snapshots would divide by
  // their square roots); r = 0 when the centred snapshots vanish
  const double lmax = n > 0 ? H[order[0] * n + order[0]] : 0.0;
  int rank = 0;
  while (rank < n && H[order[rank] * n + order[rank]] > RB_RANK_TOL * lmax) ++rank;
  if (r > rank) r = rank;
  for (int i = 0; i < nlam; ++i) lambda[i] = i < n ? H[order[i] * n + order[i]] : 0.0;
  return r;
}

// Element table G of patch K from its modes Zk [nI][rmax] and means pbar
// [3][nI] (see the header comment for the P coefficients).  Whole workgroup.
__device__ void rb_g_table(const RbBuildArgs& b, int K, const double* Zk, const double* pbar) {
  const int m = b.m, n = m - 1, nI = n * n, rmax = b.rmax;
  const int PP = b.PP, KD = b.KD, NA = rb_na(rmax);
  for (int ep = threadIdx.x; ep < KD * PP; ep += blockDim.x) {
    const int e = ep / PP, pidx = ep % PP;
    double val = 0.0;
    if (e < m * m && pidx < rb_p(rmax)) {
      const int ex = e % m, ey = e / m;
      int nid[4];
      int pxs[4] = {ex, ex + 1, ex + 1, ex}, pys[4] = {ey, ey, ey + 1, ey + 1};
      for (int c = 0; c < 4; ++c) {
        const bool inner = pxs[c] > 0 && pxs[c] < m && pys[c] > 0 && pys[c] < m;
        nid[c] = inner ? (pys[c] - 1) * n + (pxs[c] - 1) : -1;
      }
      auto zeta = [&](int q, int c) { return nid[c] >= 0 ? Zk[nid[c] * rmax + q] : 0.0; };
      auto pb = [&](int l, int c) { return nid[c] >= 0 ? pbar[l * nI + nid[c]] : pcorner(l, pxs[c], pys[c], m); };
      if (pidx < NA) {
        int q = 0, rem = pidx;
        while (rem >= rmax - q) {
          rem -= rmax - q;
          ++q;
        }
        const int qp = q + rem;
        for (int al = 0; al < 4; ++al)
          for (int be = 0; be < 4; ++be) val += zeta(q, al) * kref(al, be) * zeta(qp, be);
      } else if (pidx < NA + 3 * rmax) {
        const int l = (pidx - NA) / rmax, q = (pidx - NA) % rmax;
        for (int al = 0; al < 4; ++al)
          for (int be = 0; be < 4; ++be) val += zeta(q, al) * kref(al, be) * pb(l, be);
      } else {
        const int t = pidx - NA - 3 * rmax;
        const int ls[6] = {0, 0, 0, 1, 1, 2}, lps[6] = {0, 1, 2, 1, 2, 2};
        for (int al = 0; al < 4; ++al)
          for (int be = 0; be < 4; ++be) val += pb(ls[t], al) * kref(al, be) * pb(lps[t], be);
      }
    }
    b.G64[((int64_t)K * KD + e) * PP + pidx] = val;
    b.G32[((int64_t)K * KD + e) * PP + pidx] = (float)val;
  }
}

// Training means of the coefficient (abar, m*m values) and of the snapshots
// (phibar).  Whole workgroup.
template <typename TA>
__device__ void rb_means(const RbBuildArgs& b, int K, double* abar, double* pbar) {
  const int m = b.m, nI = (m - 1) * (m - 1), Mc = b.ncx * b.ncy;
  const int kx = K % b.ncx, ky = K / b.ncx;
  const int64_t lda = (int64_t)b.ncx * m;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int ex = e % m, ey = e / m;
    double acc = 0.0;
    for (int s = 0; s < b.ntrain; ++s) {
      const TA* a = (const TA*)b.a + (int64_t)s * (b.ncy * m) * lda;
      acc += ld(a, (int64_t)(ky * m + ey) * lda + kx * m + ex);
    }
    abar[e] = acc / b.ntrain;
  }
  for (int i = threadIdx.x; i < 3 * nI; i += blockDim.x) {
    double acc = 0.0;
    for (int s = 0; s < b.ntrain; ++s) acc += b.phi[((int64_t)s * Mc + K) * 3 * nI + i];
    pbar[i] = acc / b.ntrain;
  }
}

// The 9-point row of K_II(abar) at interior node r: diagonal in ks[8]'s
// companion kc, the eight neighbour couplings ks[q] at offsets (dxs, dys).
struct Stencil9 {
  double kc, ks[8];
};
__device__ constexpr int RB_DX[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
__device__ constexpr int RB_DY[8] = {0, 0, -1, 1, -1, -1, 1, 1};
__device__ __forceinline__ Stencil9 rb_stencil(const double* abar, int m, int ix, int iy) {
  const double aSW = abar[iy * m + ix], aSE = abar[iy * m + ix + 1];
  const double aNW = abar[(iy + 1) * m + ix], aNE = abar[(iy + 1) * m + ix + 1];
  Stencil9 st;
  st.kc = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
  st.ks[0] = -(aSW + aNW) / 6.0;
  st.ks[1] = -(aSE + aNE) / 6.0;
  st.ks[2] = -(aSW + aSE) / 6.0;
  st.ks[3] = -(aNW + aNE) / 6.0;
  st.ks[4] = -aSW / 3.0;
  st.ks[5] = -aSE / 3.0;
  st.ks[6] = -aNW / 3.0;
  st.ks[7] = -aNE / 3.0;
  return st;
}

// Primal form (3 ntrain >= nI), one workgroup per patch: the nI x nI
// snapshot Gram H = Psi Psi^T, E = K_II(abar) = L_E L_E^T (dense), the KL
// matrix C = L_E^T H L_E, its eigenpairs, modes Z = L_E^{-T} V_r.
template <typename TA>
__global__ __launch_bounds__(RB_THREADS) void rb_build_kernel(RbBuildArgs b) {
  const int K = blockIdx.x;
  const int m = b.m, n = m - 1, nI = n * n, Mc = b.ncx * b.ncy, rmax = b.rmax;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* H = b.work + (int64_t)K * 4 * nI * nI;  // snapshot Gram, then C
  double* E = H + nI * nI;                        // energy matrix, then its Cholesky factor L_E
  double* V = E + nI * nI;                        // eigenvectors
  double* T = V + nI * nI;                        // scratch
  double* pbar = b.phibar + (int64_t)K * 3 * nI;
  __shared__ double abar[64 * 64];
  __shared__ double rot[3];
  __shared__ double red[RB_THREADS];
  __shared__ int order[RB_NMAX];
  __shared__ int rsel;

  // 1. training means of the coefficient and of the snapshots
  rb_means<TA>(b, K, abar, pbar);
  __syncthreads();
  // 2. H = sum over centred snapshots (all samples, l = 0..2)
  for (int ij = tid; ij < nI * nI; ij += nt) {
    const int i = ij / nI, j = ij % nI;
    if (j < i) continue;
    double acc = 0.0;
    for (int s = 0; s < b.ntrain; ++s) {
      const double* ph = b.phi + ((int64_t)s * Mc + K) * 3 * nI;
      for (int l = 0; l < 3; ++l) acc += (ph[l * nI + i] - pbar[l * nI + i]) * (ph[l * nI + j] - pbar[l * nI + j]);
    }
    H[i * nI + j] = acc;
    H[j * nI + i] = acc;
  }
  // 3. E = K_II(abar), dense
  for (int ij = tid; ij < nI * nI; ij += nt) E[ij] = 0.0;
  __syncthreads();
  for (int r = tid; r < nI; r += nt) {
    const int ix = r % n, iy = r / n, px = ix + 1, py = iy + 1;
    const Stencil9 st = rb_stencil(abar, m, ix, iy);
    E[r * nI + r] = st.kc;
    for (int q = 0; q < 8; ++q) {
      const int qx = px + RB_DX[q], qy = py + RB_DY[q];
      if (qx >= 1 && qx <= n && qy >= 1 && qy <= n) E[r * nI + (qy - 1) * n + (qx - 1)] = st.ks[q];
    }
  }
  __syncthreads();
  // 4. E = L_E L_E^T in place (lower triangle), right looking
  for (int j = 0; j < nI; ++j) {
    if (tid == 0) E[j * nI + j] = sqrt(E[j * nI + j]);
    __syncthreads();
    const double ljj = E[j * nI + j];
    for (int i = j + 1 + tid; i < nI; i += nt) E[i * nI + j] /= ljj;
    __syncthreads();
    for (int ik = tid; ik < (nI - j - 1) * (nI - j - 1); ik += nt) {
      const int i = j + 1 + ik / (nI - j - 1), k = j + 1 + ik % (nI - j - 1);
      if (k <= i) E[i * nI + k] -= E[i * nI + j] * E[k * nI + j];
    }
    __syncthreads();
  }
  // 5. C = L_E^T H L_E  (T = H L_E, then C = L_E^T T, stored in H)
  for (int ij = tid; ij < nI * nI; ij += nt) {
    const int i = ij / nI, j = ij % nI;
    double acc = 0.0;
    for (int k = j; k < nI; ++k) acc += H[i * nI + k] * E[k * nI + j];
    T[ij] = acc;
  }
  __syncthreads();
  for (int ij = tid; ij < nI * nI; ij += nt) {
    const int i = ij / nI, j = ij % nI;
    double acc = 0.0;
    for (int k = i; k < nI; ++k) acc += E[k * nI + i] * T[k * nI + j];
    H[ij] = acc;
  }
  __syncthreads();
  // 6. eigenpairs of C
  rb_jacobi(H, V, nI, b.max_sweeps, red, rot);
  // 7. eigenvalues in descending order and the tail rule
  if (tid == 0) {
    rsel = rb_sort_tail(H, nI, order, b.tail_tol, b.rcap, rmax, b.lambda + (int64_t)K * nI, nI);
    b.rK[K] = rsel;
  }
  __syncthreads();
  const int r = rsel;
  // 8. Z = L_E^{-T} V_r (backward substitution per column), zero beyond r
  double* Zk = b.Z + (int64_t)K * nI * rmax;
  for (int q = tid; q < rmax; q += nt) {
    if (q >= r) {
      for (int i = 0; i < nI; ++i) Zk[i * rmax + q] = 0.0;
      continue;
    }
    const int col = order[q];
    for (int i = nI - 1; i >= 0; --i) {
      double v = V[i * nI + col];
      for (int k = i + 1; k < nI; ++k) v -= E[k * nI + i] * Zk[k * rmax + q];
      Zk[i * rmax + q] = v / E[i * nI + i];
    }
  }
  __syncthreads();
  // 9. element table G
  rb_g_table(b, K, Zk, pbar);
}

// Dual form, the method of snapshots (3 ntrain < nI): with Psi the nI x ns
// matrix of centred snapshots (ns = 3 ntrain, column c = 3 s + l), the KL
// expansion in the energy inner product of E = K_II(abar) is the
// eigen-decomposition of the ns x ns Gram matrix C = Psi^T E Psi = V Lambda
// V^T (the same nonzero eigenvalues as the primal C = L_E^T Psi Psi^T L_E),
// and the modes are z_q = Psi v_q / sqrt(lambda_q), so that Z^T E Z = I.
// Three steps over the patches: W = E Psi (work layout [K][c][i]), the Gram
// C = Psi^T W in 64 x 64 tiles, then per patch the eigenpairs, modes and G.
struct RbDual {
  int ns;
  double* abar;  // [M][m*m]
  double* W;     // [M][ns][nI]
  double* C;     // [M][ns][ns]
  double* V;     // [M][ns][ns]
};

__device__ __forceinline__ double rb_psi(const RbBuildArgs& b, int K, int c, int i, int nI) {
  const int s = c / 3, l = c - 3 * (c / 3);
  const int Mc = b.ncx * b.ncy;
  return b.phi[(((int64_t)s * Mc + K) * 3 + l) * nI + i] - b.phibar[((int64_t)K * 3 + l) * nI + i];
}

template <typename TA>
__global__ __launch_bounds__(RB_THREADS) void rb_dual_means_kernel(RbBuildArgs b, RbDual d) {
  const int K = blockIdx.x, m = b.m, nI = (m - 1) * (m - 1);
  rb_means<TA>(b, K, d.abar + (int64_t)K * m * m, b.phibar + (int64_t)K * 3 * nI);
}

// W[c][i] = (E Psi)_{i c}: one thread per interior node i, all columns c.
__global__ __launch_bounds__(RB_THREADS) void rb_dual_energy_kernel(RbBuildArgs b, RbDual d) {
  const int K = blockIdx.y, m = b.m, n = m - 1, nI = n * n;
  const int i = blockIdx.x * RB_THREADS + threadIdx.x;
  if (i >= nI) return;
  const int ix = i % n, iy = i / n, px = ix + 1, py = iy + 1;
  const Stencil9 st = rb_stencil(d.abar + (int64_t)K * m * m, m, ix, iy);
  int nb[8];
  for (int q = 0; q < 8; ++q) {
    const int qx = px + RB_DX[q], qy = py + RB_DY[q];
    nb[q] = (qx >= 1 && qx <= n && qy >= 1 && qy <= n) ? (qy - 1) * n + (qx - 1) : -1;
  }
  double* W = d.W + (int64_t)K * d.ns * nI;
  for (int c = 0; c < d.ns; ++c) {
    double v = st.kc * rb_psi(b, K, c, i, nI);
    for (int q = 0; q < 8; ++q)
      if (nb[q] >= 0) v += st.ks[q] * rb_psi(b, K, c, nb[q], nI);
    W[(int64_t)c * nI + i] = v;
  }
}

// C = Psi^T W in 64 x 64 tiles (upper tiles computed, mirrored): the k loop
// over the interior nodes in chunks of 32 staged in LDS; each thread
// accumulates a 4 x 4 block of the tile.
constexpr int RBG_T = 64, RBG_K = 32;
__global__ __launch_bounds__(RB_THREADS) void rb_dual_gram_kernel(RbBuildArgs b, RbDual d) {
  const int K = blockIdx.y, m = b.m, nI = (m - 1) * (m - 1), ns = d.ns;
  const int nt = (ns + RBG_T - 1) / RBG_T;
  int t = blockIdx.x, tc = 0;
  while (t >= nt - tc) {  // upper-triangle tile index -> (tc, td), tc <= td
    t -= nt - tc;
    ++tc;
  }
  const int td = tc + t;
  __shared__ double Ps[RBG_K][RBG_T + 1], Ws[RBG_K][RBG_T + 1];
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  const double* W = d.W + (int64_t)K * ns * nI;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < nI; k0 += RBG_K) {
    for (int idx = tid; idx < RBG_K * RBG_T; idx += RB_THREADS) {
      const int kk = idx % RBG_K, cc = idx / RBG_K;
      const int c = tc * RBG_T + cc, dd = td * RBG_T + cc, i = k0 + kk;
      Ps[kk][cc] = (c < ns && i < nI) ? rb_psi(b, K, c, i, nI) : 0.0;
      Ws[kk][cc] = (dd < ns && i < nI) ? W[(int64_t)dd * nI + i] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < RBG_K; ++kk) {
      double pv[4], wv[4];
      for (int u = 0; u < 4; ++u) {
        pv[u] = Ps[kk][4 * ty + u];
        wv[u] = Ws[kk][4 * tx + u];
      }
      for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) acc[u][v] += pv[u] * wv[v];
    }
    __syncthreads();
  }
  double* C = d.C + (int64_t)K * ns * ns;
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) {
      const int c = tc * RBG_T + 4 * ty + u, dd = td * RBG_T + 4 * tx + v;
      if (c < ns && dd < ns) {
        C[(int64_t)c * ns + dd] = acc[u][v];
        if (tc != td) C[(int64_t)dd * ns + c] = acc[u][v];
      }
    }
}

// Per patch: eigenpairs of C, the tail rule, modes z_q = Psi v_q /
// sqrt(lambda_q) (zero beyond r), the element table.
__global__ __launch_bounds__(RB_THREADS) void rb_dual_finish_kernel(RbBuildArgs b, RbDual d) {
  const int K = blockIdx.x, m = b.m, nI = (m - 1) * (m - 1), ns = d.ns, rmax = b.rmax;
  __shared__ double rot[3];
  __shared__ double red[RB_THREADS];
  __shared__ int order[RB_NMAX];
  __shared__ int rsel;
  double* C = d.C + (int64_t)K * ns * ns;
  double* V = d.V + (int64_t)K * ns * ns;
  rb_jacobi(C, V, ns, b.max_sweeps, red, rot);
  if (threadIdx.x == 0) {
    rsel = rb_sort_tail(C, ns, order, b.tail_tol, b.rcap, rmax, b.lambda + (int64_t)K * nI, nI);
    b.rK[K] = rsel;
  }
  __syncthreads();
  const int r = rsel;
  double* Zk = b.Z + (int64_t)K * nI * rmax;
  for (int iq = threadIdx.x; iq < nI * rmax; iq += blockDim.x) {
    const int i = iq / rmax, q = iq % rmax;
    double v = 0.0;
    if (q < r) {
      const int col = order[q];
      const double lam = C[col * ns + col];
      for (int c = 0; c < ns; ++c) v += rb_psi(b, K, c, i, nI) * V[(int64_t)c * ns + col];
      v = lam > 0.0 ? v / sqrt(lam) : 0.0;
    }
    Zk[iq] = v;
  }
  __syncthreads();
  rb_g_table(b, K, Zk, b.phibar + (int64_t)K * 3 * nI);
}

int64_t rb_work_doubles(int ncx, int ncy, int m, int ntrain) {
  const int64_t Mc = (int64_t)ncx * ncy, nI = (int64_t)(m - 1) * (m - 1), ns = 3 * (int64_t)ntrain;
  if (ns < nI) return Mc * ((int64_t)m * m + ns * nI + 2 * ns * ns);
  return Mc * 4 * nI * nI;
}

bool rb_dual(int m, int ntrain) { return 3 * ntrain < (m - 1) * (m - 1); }

hipError_t launch_rb_build(const RbBuildArgs& b, hipStream_t st) {
  const int Mc = b.ncx * b.ncy, m = b.m, nI = (m - 1) * (m - 1);
  if (!rb_dual(m, b.ntrain)) {
    if (nI > RB_NMAX) return hipErrorInvalidValue;
    if (b.a_dtype == STOMSFEM_F32)
      hipLaunchKernelGGL(rb_build_kernel<float>, dim3(Mc), dim3(RB_THREADS), 0, st, b);
    else
      hipLaunchKernelGGL(rb_build_kernel<double>, dim3(Mc), dim3(RB_THREADS), 0, st, b);
    return hipGetLastError();
  }
  RbDual d{};
  d.ns = 3 * b.ntrain;
  if (d.ns > RB_NMAX) return hipErrorInvalidValue;
  d.abar = b.work;
  d.W = d.abar + (int64_t)Mc * m * m;
  d.C = d.W + (int64_t)Mc * d.ns * nI;
  d.V = d.C + (int64_t)Mc * d.ns * d.ns;
  if (b.a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(rb_dual_means_kernel<float>, dim3(Mc), dim3(RB_THREADS), 0, st, b, d);
  else
    hipLaunchKernelGGL(rb_dual_means_kernel<double>, dim3(Mc), dim3(RB_THREADS), 0, st, b, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rb_dual_energy_kernel, dim3((nI + RB_THREADS - 1) / RB_THREADS, Mc), dim3(RB_THREADS), 0, st, b,
                     d);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nt = (d.ns + RBG_T - 1) / RBG_T;
  hipLaunchKernelGGL(rb_dual_gram_kernel, dim3(nt * (nt + 1) / 2, Mc), dim3(RB_THREADS), 0, st, b, d);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rb_dual_finish_kernel, dim3(Mc), dim3(RB_THREADS), 0, st, b, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Online stage
// ---------------------------------------------------------------------------
// r x r LDL^T of A (packed upper in v), forward solves with the three Fh
// columns, S_ll' = B_ll' - Fh_l . A^{-1} Fh_l' = B_ll' - sum_i y_l[i] y_l'[i] / d_i
// with L y_l = Fh_l (unit L), in the arithmetic of T (FP64 for the reference
// stage, FP32 after the FP32 matrix-core products: A is close to the
// identity, since the modes are orthonormal in the energy of the training
// mean).  No square roots, and one reciprocal per pivot (FP32: the hardware
// reciprocal, within an ulp, far below the FP32 products' error).  Returns
// false on a non-positive pivot.
template <typename T>
__device__ __forceinline__ T rb_recip(T d) {
  return T(1) / d;
}
template <>
__device__ __forceinline__ float rb_recip<float>(float d) {
  return __builtin_amdgcn_rcpf(d);
}
template <int RMAX, typename T>
__device__ __forceinline__ bool rb_small_solve(const T* v, int r, double S3[3][3]) {
  constexpr int NA = RMAX * (RMAX + 1) / 2;
  T L[RMAX][RMAX];  // lower part: A, then the unit factor's l_ij (i > j)
  T U[RMAX][RMAX];  // u_ij = l_ij d_j (i > j)
  T dinv[RMAX];
  T X[3][RMAX];
  bool ok = true;
#pragma unroll
  for (int q = 0; q < RMAX; ++q)
#pragma unroll
    for (int qp = q; qp < RMAX; ++qp) {
      // identity on the unused modes keeps the factorisation well defined
      const T a = v[q * RMAX - q * (q - 1) / 2 + (qp - q)];
      L[qp][q] = (q < r && qp < r) ? a : (q == qp ? T(1) : T(0));
    }
  // Crout LDL^T: u_ij = a_ij - sum_k u_ik l_jk, d_j = a_jj - sum_k u_jk l_jk
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    T d = L[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= U[j][k] * L[j][k];
    ok = ok && d > T(0);
    const T inv = rb_recip<T>(d);
    dinv[j] = inv;
#pragma unroll
    for (int i = j + 1; i < RMAX; ++i) {
      T u = L[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) u -= U[i][k] * L[j][k];
      U[i][j] = u;
      L[i][j] = u * inv;
    }
  }
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
      T t = (i < r) ? v[NA + l * RMAX + i] : T(0);
#pragma unroll
      for (int k = 0; k < i; ++k) t -= L[i][k] * X[l][k];
      X[l][i] = t;
    }
  const int ls[6] = {0, 0, 0, 1, 1, 2}, lps[6] = {0, 1, 2, 1, 2, 2};
  T Z[3][RMAX];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int i = 0; i < RMAX; ++i) Z[l][i] = X[l][i] * dinv[i];
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    T acc = v[NA + 3 * RMAX + t];
#pragma unroll
    for (int i = 0; i < RMAX; ++i) acc -= Z[ls[t]][i] * X[lps[t]][i];
    S3[ls[t]][lps[t]] = (double)acc;
    S3[lps[t]][ls[t]] = (double)acc;
  }
  return ok;
}

// FP64 reference online stage: one thread per pair, dot products with G64.
template <int RMAX, typename TA>
__global__ __launch_bounds__(64) void rb_apply_f64_kernel(RbApplyArgs ra) {
  const UpArgs& args = ra.up;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= args.npairs) return;
  const int m = args.m, Mc = args.ncx * args.ncy;
  const int64_t s = p / Mc;
  const int K = (int)(p - s * Mc);
  const TA* a = (const TA*)args.a + block_offset(s, K, args.ncx, args.ncy, m);
  const int64_t lda = (int64_t)args.ncx * m;
  constexpr int P = RMAX * (RMAX + 1) / 2 + 3 * RMAX + 6;
  double v[P];
#pragma unroll
  for (int q = 0; q < P; ++q) v[q] = 0.0;
  const double* G = ra.G64 + (int64_t)K * ra.KD * ra.PP;
  for (int e = 0; e < m * m; ++e) {
    const double ae = ld(a, (e / m) * lda + (e % m));
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] += ae * G[e * ra.PP + q];
  }
  double S3[3][3];
  const bool ok = rb_small_solve<RMAX, double>(v, ra.rK[K], S3);
  store_packed(args.S + p * 10, S3);
  if (args.status) args.status[p] = ok ? STOMSFEM_OK : STOMSFEM_ENOTSPD;
}

// FP32 MFMA online stage.  Workgroup = 4 wavefronts = 128 samples of one
// patch.  C[128 x PP] = A[128 x KD] G[KD x PP] with v_mfma_f32_16x16x4f32 and
// FP32 accumulation (wavefront w computes rows 32w..32w+31, two row tiles,
// all PP/16 column tiles), the k dimension (the patch's m*m fine elements,
// padded to KD, a multiple of 64) in chunks of 64 staged in LDS: the chunk's
// coefficients of the 128 samples and its 64 rows of the patch's table,
// the next chunk's coefficients loaded into registers while the current one
// is multiplied.  Then one lane per sample does the FP32 r x r solve (the
// result rows pass through LDS, in the space of the staging buffers).
constexpr int RBA_SAMPLES = 128;
constexpr int RBA_KC = 64;
constexpr int RBA_LDA = RBA_KC + 4;
constexpr int RBA_PF = RBA_SAMPLES * RBA_KC / 256;  // coefficients per thread and chunk

// Workgroup order: one-dimensional grid of ntiles x M workgroups.  When a
// patch's coefficient row is shorter than a 128-byte cache line, the patch
// index runs fastest, so that neighbouring patches, which share the lines of
// a sample, are read by one L2: the hardware deals consecutive workgroups
// round-robin to the eight XCDs (each with its own L2), and the logical index
// L = (b mod 8) (n / 8) + b / 8 gives each XCD a contiguous range.
// Otherwise the sample tile runs fastest and consecutive workgroups share
// the patch's table.
//
// OS = true: the oversampled patches (rb_os.hip).  The block of element K is
// its patch (side m + 2 os_o, origin rbo_origin), the table is GO32 (PP =
// RBO_PO columns: A, Fh and the element sums U), and the per-sample epilogue
// is the FP64 solve for c and the recombination at K's corners (16 entries
// per pair).  vec_ok: every patch row starts on a 16-byte boundary.
//
// MT = true (plain variant, single-chunk tiles): a workgroup takes tpw
// consecutive sample tiles of its patch and the (tile, chunk) steps form one
// loop, so the next tile's coefficients are in flight during the current
// tile's products and solves (two wavefronts per SIMD kept for the extra
// prefetch registers).  MT = false: one tile per workgroup (tpw = 1).
template <int RMAX, int PP, typename TA, bool OS = false, bool MT = false>
__global__ __launch_bounds__(256, MT ? 2 : 1) void rb_apply_mfma_kernel(RbApplyArgs ra, int64_t ntiles,
                                                                       int patch_fast, int vec_ok, int tpw) {
  using f4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
  const UpArgs& args = ra.up;
  const int m = args.m, Mc = args.ncx * args.ncy, KD = ra.KD;
  const int bs = OS ? m + 2 * ra.os_o : m, mm = bs * bs;  // block side and elements
  const int64_t ngroups = (ntiles + tpw - 1) / tpw, nb = ngroups * Mc, b = blockIdx.x;
  const int64_t L = (patch_fast && nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int K = (int)(patch_fast ? L % Mc : L / ngroups);
  const int64_t tile0 = (patch_fast ? L / Mc : L % ngroups) * tpw;
  const int64_t lda = (int64_t)args.ncx * m;
  constexpr int AS_FLOATS = RBA_SAMPLES * RBA_LDA, GS_FLOATS = RBA_KC * PP;
  constexpr int CS_FLOATS = RBA_SAMPLES * (PP + 1);
  constexpr int SM_FLOATS = (AS_FLOATS + GS_FLOATS) > CS_FLOATS ? (AS_FLOATS + GS_FLOATS) : CS_FLOATS;
  __shared__ __align__(16) float smem[SM_FLOATS];
  float(*As)[RBA_LDA] = reinterpret_cast<float(*)[RBA_LDA]>(smem);
  float(*Gs)[PP] = reinterpret_cast<float(*)[PP]>(smem + AS_FLOATS);
  float(*Cs)[PP + 1] = reinterpret_cast<float(*)[PP + 1]>(smem);
  const int tid = threadIdx.x;
  const int kx = K % args.ncx, ky = K / args.ncx;
  const int bx0 = OS ? rbo_origin(kx, m, ra.os_o, args.ncx * m) : kx * m;
  const int by0 = OS ? rbo_origin(ky, m, ra.os_o, args.ncy * m) : ky * m;
  const int w = tid / 64, lane = tid % 64;
  constexpr int NTILE = PP / 16;
  f4 acc[2][NTILE];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int t = 0; t < NTILE; ++t) acc[h][t] = f4{0.f, 0.f, 0.f, 0.f};
  const float* G = ra.G32 + (int64_t)K * KD * PP;
  // thread tid loads coefficient (i, e0 + c) of the tile starting at sample
  // s0 for idx = tid + 256 q, i = idx / KC
  auto load_chunk = [&](int64_t s0, int e0, float (&v)[RBA_PF]) {
#pragma unroll
    for (int q = 0; q < RBA_PF; ++q) {
      const int idx = tid + 256 * q, i = idx / RBA_KC, e = e0 + idx % RBA_KC;
      const int64_t s = s0 + i;
      float x = 0.0f;
      if (s < args.nsamples && e < mm) {
        const TA* a = (const TA*)args.a + s * (int64_t)(args.ncy * m) * lda;
        x = (float)ld(a, (int64_t)(by0 + e / bs) * lda + bx0 + e % bs);
      }
      v[q] = x;
    }
  };
  // block side in {8, 16, 32} with FP32 coefficients: a chunk of 64
  // elements is 64 / bs whole rows of the block, so each sample's share comes
  // in 16-byte loads (16 per sample and chunk: thread tid takes float4
  // f = idx % 16 of sample idx / 16, idx = tid + 256 q)
  const bool vec = std::is_same<TA, float>::value && vec_ok && (bs == 8 || bs == 16 || bs == 32);
  const int lm = bs == 8 ? 3 : bs == 16 ? 4 : 5;
  auto load_chunk_vec = [&](int64_t s0, int e0, float (&v)[RBA_PF]) {
#pragma unroll
    for (int q = 0; q < RBA_PF / 4; ++q) {
      const int idx = tid + 256 * q, i = idx >> 4, e = e0 + 4 * (idx & 15);
      const int64_t s = s0 + i;
      f4 x = f4{0.f, 0.f, 0.f, 0.f};
      if (s < args.nsamples && e < mm) {
        const float* a = (const float*)args.a + s * (int64_t)(args.ncy * m) * lda;
        x = *reinterpret_cast<const f4*>(a + (int64_t)(by0 + (e >> lm)) * lda + bx0 + (e & (bs - 1)));
      }
      v[4 * q] = x[0];
      v[4 * q + 1] = x[1];
      v[4 * q + 2] = x[2];
      v[4 * q + 3] = x[3];
    }
  };
  const int nch = KD / RBA_KC, nit = (MT ? tpw : 1) * nch;
  auto load_step = [&](int it, float (&v)[RBA_PF]) {
    const int64_t s0 = (tile0 + it / nch) * RBA_SAMPLES;
    const int e0 = (it % nch) * RBA_KC;
    if (vec)
      load_chunk_vec(s0, e0, v);
    else
      load_chunk(s0, e0, v);
  };
  float pf[RBA_PF];
  // one (tile, chunk) step: stage the coefficients and the table chunk, start
  // the next step's loads, accumulate the products
  auto step = [&](int it) {
    const int e0 = (it % nch) * RBA_KC;
    __syncthreads();  // the previous step's readers (products or solves) are done
    if (vec) {
#pragma unroll
      for (int q = 0; q < RBA_PF / 4; ++q) {
        const int idx = tid + 256 * q;
        *reinterpret_cast<f4*>(&As[idx >> 4][4 * (idx & 15)]) =
            f4{pf[4 * q], pf[4 * q + 1], pf[4 * q + 2], pf[4 * q + 3]};
      }
    } else {
#pragma unroll
      for (int q = 0; q < RBA_PF; ++q) {
        const int idx = tid + 256 * q;
        As[idx / RBA_KC][idx % RBA_KC] = pf[q];
      }
    }
    // the chunk's 64 table rows: contiguous, PP a multiple of 4, 16-byte loads
    static_assert(PP % 4 == 0 && (RBA_KC * PP) % (4 * 256) == 0, "table chunk in float4 per thread");
#pragma unroll
    for (int q = 0; q < RBA_KC * PP / (4 * 256); ++q) {
      const int idx = 4 * (tid + 256 * q);
      *reinterpret_cast<f4*>(&Gs[0][0] + idx) = *reinterpret_cast<const f4*>(G + (int64_t)e0 * PP + idx);
    }
    __syncthreads();
    if (it + 1 < nit) load_step(it + 1, pf);  // in flight during the products (and the solves)
#pragma unroll 4
    for (int kk = 0; kk < RBA_KC / 4; ++kk) {
      const float av0 = As[32 * w + (lane & 15)][4 * kk + (lane >> 4)];
      const float av1 = As[32 * w + 16 + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
      for (int t = 0; t < NTILE; ++t) {
        const float bv = Gs[4 * kk + (lane >> 4)][16 * t + (lane & 15)];
        acc[0][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av0, bv, acc[0][t], 0, 0, 0);
        acc[1][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av1, bv, acc[1][t], 0, 0, 0);
      }
    }
  };
  // a complete tile: its rows through LDS, then one lane per sample
  auto finish_tile = [&](int64_t tile) {
    __syncthreads();  // Cs overlays the staging buffers
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int t = 0; t < NTILE; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Cs[32 * w + 16 * h + 4 * (lane >> 4) + v][16 * t + (lane & 15)] = acc[h][t][v];
        acc[h][t] = f4{0.f, 0.f, 0.f, 0.f};
      }
    __syncthreads();
    const int64_t s = tile * RBA_SAMPLES + tid;
    if (tid < RBA_SAMPLES && s < args.nsamples) {
      const int64_t p = s * Mc + K;
      if constexpr (OS) {
        double c[3][RMAX];
        const bool ok = rbo_coeffs<RMAX>(&Cs[tid][0], ra.rK[K], c);
        double S[4][4];
        const bool nonsing = rbo_recombine<RMAX>(c, &Cs[tid][RBO_H], ra.Pc + (int64_t)K * 4 * RBO_NF, S);
        double* out = args.S + p * 16;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int lp = 0; lp < 4; ++lp) out[4 * i + lp] = S[i][lp];
        if (args.status) args.status[p] = (ok && nonsing) ? STOMSFEM_OK : STOMSFEM_ENOTSPD;
      } else {
        constexpr int P = RMAX * (RMAX + 1) / 2 + 3 * RMAX + 6;
        float v[P];
#pragma unroll
        for (int q = 0; q < P; ++q) v[q] = Cs[tid][q];
        double S3[3][3];
        const bool ok = rb_small_solve<RMAX, float>(v, ra.rK[K], S3);
        store_packed(args.S + p * 10, S3);
        if (args.status) args.status[p] = ok ? STOMSFEM_OK : STOMSFEM_ENOTSPD;
      }
    }
  };
  load_step(0, pf);
  if constexpr (!MT) {
    for (int it = 0; it < nch; ++it) step(it);
    finish_tile(tile0);
  } else {
    for (int it = 0; it < nit; ++it) {
      step(it);
      if (it % nch == nch - 1) finish_tile(tile0 + it / nch);
    }
  }
}

// Tiles per workgroup.  Where a tile is a single chunk (m <= 8) nothing
// overlaps its loads otherwise: about four workgroups per CU (1024) when the
// batch has that many tiles, at most eight tiles each (8x8 mesh, 16 384
// samples: 0.205 ms with one tile per workgroup, 0.175 ms with four, 0.170 ms
// with eight).  Longer tiles already overlap chunk with chunk, and grouping
// them only costs parallelism (32x32 mesh, H/h = 32: 6.2 ms with one, 6.8 ms
// with eight).
static int rba_tiles_per_workgroup(int64_t ntiles, int Mc, int KD) {
  if (KD > RBA_KC) return 1;
  const int64_t t = ntiles * Mc / 1024;
  return (int)(t < 1 ? 1 : t > 8 ? 8 : t);
}

int rb_pad_p(int rmax) { return ((rb_p(rmax) + 15) / 16) * 16; }
int rb_pad_kd(int m) { return ((m * m + RBA_KC - 1) / RBA_KC) * RBA_KC; }

hipError_t launch_rb_apply(const RbApplyArgs& ra, int a_dtype, bool f64, hipStream_t st) {
  const UpArgs& u = ra.up;
  if (u.npairs == 0) return hipSuccess;
  if (ra.rmax != 8) return hipErrorInvalidValue;
  if (f64) {
    const int64_t blocks = (u.npairs + 63) / 64;
    if (a_dtype == STOMSFEM_F32)
      hipLaunchKernelGGL((rb_apply_f64_kernel<8, float>), dim3((unsigned)blocks), dim3(64), 0, st, ra);
    else
      hipLaunchKernelGGL((rb_apply_f64_kernel<8, double>), dim3((unsigned)blocks), dim3(64), 0, st, ra);
    return hipGetLastError();
  }
  if (ra.PP != 80 || ra.KD % RBA_KC != 0 || ra.KD < u.m * u.m) return hipErrorInvalidValue;
  const int Mc = u.ncx * u.ncy;
  const int64_t ntiles = (u.nsamples + RBA_SAMPLES - 1) / RBA_SAMPLES;
  const int tpw = rba_tiles_per_workgroup(ntiles, Mc, ra.KD);
  const int64_t nb = (ntiles + tpw - 1) / tpw * Mc;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  const int elem = a_dtype == STOMSFEM_F32 ? 4 : 8;
  const int patch_fast = u.m * elem < 128 ? 1 : 0;
  // single-chunk tiles take the multi-tile variant
  if (ra.KD == RBA_KC) {
    if (a_dtype == STOMSFEM_F32)
      hipLaunchKernelGGL((rb_apply_mfma_kernel<8, 80, float, false, true>), dim3((unsigned)nb), dim3(256), 0, st, ra,
                         ntiles, patch_fast, 1, tpw);
    else
      hipLaunchKernelGGL((rb_apply_mfma_kernel<8, 80, double, false, true>), dim3((unsigned)nb), dim3(256), 0, st,
                         ra, ntiles, patch_fast, 1, tpw);
  } else {
    if (a_dtype == STOMSFEM_F32)
      hipLaunchKernelGGL((rb_apply_mfma_kernel<8, 80, float>), dim3((unsigned)nb), dim3(256), 0, st, ra, ntiles,
                         patch_fast, 1, tpw);
    else
      hipLaunchKernelGGL((rb_apply_mfma_kernel<8, 80, double>), dim3((unsigned)nb), dim3(256), 0, st, ra, ntiles,
                         patch_fast, 1, tpw);
  }
  return hipGetLastError();
}

hipError_t launch_rb_os_apply_mfma(const RbApplyArgs& ra, int a_dtype, hipStream_t st) {
  const UpArgs& u = ra.up;
  if (u.npairs == 0) return hipSuccess;
  const int bs = u.m + 2 * ra.os_o;
  if (ra.rmax != 8 || ra.PP != RBO_PO || ra.KD % RBA_KC != 0 || ra.KD < bs * bs || !ra.Pc)
    return hipErrorInvalidValue;
  const int Mc = u.ncx * u.ncy;
  const int64_t ntiles = (u.nsamples + RBA_SAMPLES - 1) / RBA_SAMPLES;
  const int tpw = 1;  // one tile per workgroup (the kernel's OS variant)
  const int64_t nb = ntiles * Mc;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  const int elem = a_dtype == STOMSFEM_F32 ? 4 : 8;
  const int patch_fast = bs * elem < 128 ? 1 : 0;
  // patch rows on 16-byte boundaries: every origin is a multiple of 4 cells
  const int vec_ok = (u.m % 4 == 0 && ra.os_o % 4 == 0 && (u.ncx * u.m) % 4 == 0) ? 1 : 0;
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL((rb_apply_mfma_kernel<8, RBO_PO, float, true>), dim3((unsigned)nb), dim3(256), 0, st, ra,
                       ntiles, patch_fast, vec_ok, tpw);
  else
    hipLaunchKernelGGL((rb_apply_mfma_kernel<8, RBO_PO, double, true>), dim3((unsigned)nb), dim3(256), 0, st, ra,
                       ntiles, patch_fast, vec_ok, tpw);
  return hipGetLastError();
}

}  // namespace stomsfem
