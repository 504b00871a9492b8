// Reduced-basis upscaling (Sec. 3.2, eqs. KLphi, localRB, localRBsystem,
// RBaffine / localAF; Algorithms 3 and 4).
//
// Offline (per patch K, from N_train coefficient samples):
//   cell_phi_kernel  -- the cell-problem solutions phi^l(xi_s), l = 0..2, on
//                       the interior nodes (banded LDL^T in LDS, one
//                       wavefront per pair, forward and backward solves);
//   rb_build_kernel  -- one workgroup per patch: mean phibar^l, centred
//                       snapshot Gram H = Psi Psi^T, energy matrix
//                       E = K_II(abar) = L_E L_E^T with abar the training mean
//                       of the coefficient, C = L_E^T H L_E (the Gram matrix of
//                       the KL expansion in the energy inner product), cyclic
//                       Jacobi eigen-decomposition C = V Lambda V^T, the tail
//                       rule for r, modes Z = L_E^{-T} V_r (Z^T E Z = I), and
//                       the element table G.
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
// Online: rb_apply_mfma_kernel (FP32 MFMA 16x16x4, FP32 accumulation, FP64
// r x r solve) and rb_apply_f64_kernel (FP64 throughout, for parity checks).
#include "rb.h"

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
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(cell_phi_kernel<float>, dim3((unsigned)blocks), dim3(64), lds, st, pa);
  else
    hipLaunchKernelGGL(cell_phi_kernel<double>, dim3((unsigned)blocks), dim3(64), lds, st, pa);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Offline build, one workgroup per patch
// ---------------------------------------------------------------------------
constexpr int RB_THREADS = 256;

template <typename TA>
__global__ __launch_bounds__(RB_THREADS) void rb_build_kernel(RbBuildArgs b) {
  const int K = blockIdx.x;
  const int m = b.m, n = m - 1, nI = n * n, Mc = b.ncx * b.ncy, rmax = b.rmax;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int kx = K % b.ncx, ky = K / b.ncx;
  const int64_t lda = (int64_t)b.ncx * m;
  double* H = b.work + (int64_t)K * 4 * nI * nI;  // snapshot Gram, then C
  double* E = H + nI * nI;                        // energy matrix, then its Cholesky factor L_E
  double* V = E + nI * nI;                        // eigenvectors
  double* T = V + nI * nI;                        // scratch
  double* pbar = b.phibar + (int64_t)K * 3 * nI;
  __shared__ double abar[64 * 64];
  __shared__ double rot[3];
  __shared__ double red[RB_THREADS];
  __shared__ int order[1024];
  __shared__ int rsel;

  // 1. training means of the coefficient and of the snapshots
  for (int e = tid; e < m * m; e += nt) {
    const int ex = e % m, ey = e / m;
    double acc = 0.0;
    for (int s = 0; s < b.ntrain; ++s) {
      const TA* a = (const TA*)b.a + (int64_t)s * (b.ncy * m) * lda;
      acc += ld(a, (int64_t)(ky * m + ey) * lda + kx * m + ex);
    }
    abar[e] = acc / b.ntrain;
  }
  for (int i = tid; i < 3 * nI; i += nt) {
    double acc = 0.0;
    for (int s = 0; s < b.ntrain; ++s) acc += b.phi[((int64_t)s * Mc + K) * 3 * nI + i];
    pbar[i] = acc / b.ntrain;
  }
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
    const double aSW = abar[iy * m + ix], aSE = abar[iy * m + ix + 1];
    const double aNW = abar[(iy + 1) * m + ix], aNE = abar[(iy + 1) * m + ix + 1];
    E[r * nI + r] = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
    const int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
    const int dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
    const double ks[8] = {-(aSW + aNW) / 6.0, -(aSE + aNE) / 6.0, -(aSW + aSE) / 6.0, -(aNW + aNE) / 6.0,
                          -aSW / 3.0,         -aSE / 3.0,         -aNW / 3.0,         -aNE / 3.0};
    for (int q = 0; q < 8; ++q) {
      const int qx = px + dxs[q], qy = py + dys[q];
      if (qx >= 1 && qx <= n && qy >= 1 && qy <= n) E[r * nI + (qy - 1) * n + (qx - 1)] = ks[q];
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
  for (int ij = tid; ij < nI * nI; ij += nt) V[ij] = (ij / nI == ij % nI) ? 1.0 : 0.0;
  __syncthreads();
  // symmetrise (rounding)
  for (int ij = tid; ij < nI * nI; ij += nt) {
    const int i = ij / nI, j = ij % nI;
    if (j > i) {
      const double v = 0.5 * (H[i * nI + j] + H[j * nI + i]);
      H[i * nI + j] = v;
      H[j * nI + i] = v;
    }
  }
  __syncthreads();
  // 6. cyclic Jacobi: rotations in the (p, q) planes until the off-diagonal
  //    mass is negligible against the diagonal
  for (int sweep = 0; sweep < b.max_sweeps; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int ij = tid; ij < nI * nI; ij += nt) {
      const double v = H[ij] * H[ij];
      if (ij / nI == ij % nI) dia += v; else off += v;
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
    for (int p = 0; p < nI - 1; ++p)
      for (int q = p + 1; q < nI; ++q) {
        if (tid == 0) {
          const double apq = H[p * nI + q];
          double c = 1.0, s = 0.0;
          if (apq != 0.0) {
            const double tau = (H[q * nI + q] - H[p * nI + p]) / (2.0 * apq);
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
          for (int k = tid; k < nI; k += nt) {
            const double hp = H[k * nI + p], hq = H[k * nI + q];
            H[k * nI + p] = c * hp - s * hq;
            H[k * nI + q] = s * hp + c * hq;
            const double vp = V[k * nI + p], vq = V[k * nI + q];
            V[k * nI + p] = c * vp - s * vq;
            V[k * nI + q] = s * vp + c * vq;
          }
          __syncthreads();
          for (int k = tid; k < nI; k += nt) {
            const double hp = H[p * nI + k], hq = H[q * nI + k];
            H[p * nI + k] = c * hp - s * hq;
            H[q * nI + k] = s * hp + c * hq;
          }
        }
        __syncthreads();
      }
  }
  // 7. eigenvalues in descending order and the tail rule
  if (tid == 0) {
    for (int i = 0; i < nI; ++i) order[i] = i;
    for (int i = 0; i < nI; ++i) {  // selection sort (nI is small)
      int best = i;
      for (int j = i + 1; j < nI; ++j)
        if (H[order[j] * nI + order[j]] > H[order[best] * nI + order[best]]) best = j;
      const int t = order[i];
      order[i] = order[best];
      order[best] = t;
    }
    double tot = 0.0;
    for (int i = 0; i < nI; ++i) tot += fmax(H[order[i] * nI + order[i]], 0.0);
    int r = nI;
    double tail = tot;
    for (int q = 1; q <= nI; ++q) {
      tail -= fmax(H[order[q - 1] * nI + order[q - 1]], 0.0);
      const double rel = tot > 0 ? sqrt(fmax(tail, 0.0) / tot) : 0.0;
      if (rel <= b.tail_tol) {
        r = q;
        break;
      }
    }
    if (r > b.rcap) r = b.rcap;
    if (r > rmax) r = rmax;
    if (r > nI) r = nI;
    rsel = r;
    b.rK[K] = r;
    for (int i = 0; i < nI; ++i) b.lambda[(int64_t)K * nI + i] = H[order[i] * nI + order[i]];
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
  const int PP = b.PP, KD = b.KD, NA = rb_na(rmax);
  for (int ep = tid; ep < KD * PP; ep += nt) {
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

hipError_t launch_rb_build(const RbBuildArgs& b, hipStream_t st) {
  const int Mc = b.ncx * b.ncy;
  if (b.a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(rb_build_kernel<float>, dim3(Mc), dim3(RB_THREADS), 0, st, b);
  else
    hipLaunchKernelGGL(rb_build_kernel<double>, dim3(Mc), dim3(RB_THREADS), 0, st, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Online stage
// ---------------------------------------------------------------------------
// r x r Cholesky of A (packed upper in v), solves with the three Fh columns,
// S_ll' = B_ll' - Fh_l . A^{-1} Fh_l'.  All in FP64.  Returns false on a
// non-positive pivot.
template <int RMAX>
__device__ __forceinline__ bool rb_small_solve(const double* v, int r, double S3[3][3]) {
  constexpr int NA = RMAX * (RMAX + 1) / 2;
  double L[RMAX][RMAX];
  double X[3][RMAX];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < RMAX; ++i)
#pragma unroll
    for (int j = 0; j < RMAX; ++j) L[i][j] = 0.0;
#pragma unroll
  for (int q = 0; q < RMAX; ++q)
#pragma unroll
    for (int qp = q; qp < RMAX; ++qp) {
      const double a = v[q * RMAX - q * (q - 1) / 2 + (qp - q)];
      L[qp][q] = a;
    }
  // identity on the unused modes keeps the factorisation well defined
#pragma unroll
  for (int q = 0; q < RMAX; ++q)
    if (q >= r) {
#pragma unroll
      for (int j = 0; j < RMAX; ++j) L[q][j] = (j == q) ? 1.0 : 0.0;
#pragma unroll
      for (int i = 0; i < RMAX; ++i)
        if (i != q) L[i][q] = 0.0;
    }
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    double d = L[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    ok = ok && d > 0.0;
    const double ljj = sqrt(d);
    L[j][j] = ljj;
    const double inv = 1.0 / ljj;
#pragma unroll
    for (int i = j + 1; i < RMAX; ++i) {
      double t = L[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t * inv;
    }
  }
  // forward solves L y = Fh_l (only the forward half is needed:
  // Fh_l . A^{-1} Fh_l' = y_l . y_l')
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
      double t = (i < r) ? v[NA + l * RMAX + i] : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) t -= L[i][k] * X[l][k];
      X[l][i] = t / L[i][i];
    }
  const int ls[6] = {0, 0, 0, 1, 1, 2}, lps[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    double acc = v[NA + 3 * RMAX + t];
#pragma unroll
    for (int i = 0; i < RMAX; ++i) acc -= X[ls[t]][i] * X[lps[t]][i];
    S3[ls[t]][lps[t]] = acc;
    S3[lps[t]][ls[t]] = acc;
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
  const bool ok = rb_small_solve<RMAX>(v, ra.rK[K], S3);
  store_packed(args.S + p * 10, S3);
  if (args.status) args.status[p] = ok ? STOMSFEM_OK : STOMSFEM_ENOTSPD;
}

// FP32 MFMA online stage.  Workgroup = 4 wavefronts = 64 samples of one
// patch.  C[64 x PP] = A[64 x KD] G[KD x PP] with v_mfma_f32_16x16x4f32
// (wavefront w computes rows 16w..16w+15, all PP/16 column tiles); then one
// lane per sample does the FP64 r x r solve.
constexpr int RBA_SAMPLES = 64;

template <int RMAX, int KD, int PP, typename TA>
__global__ __launch_bounds__(256) void rb_apply_mfma_kernel(RbApplyArgs ra) {
  using f4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
  const UpArgs& args = ra.up;
  const int m = args.m, Mc = args.ncx * args.ncy;
  const int K = blockIdx.y;
  const int64_t s0 = (int64_t)blockIdx.x * RBA_SAMPLES;
  const int64_t lda = (int64_t)args.ncx * m;
  __shared__ float As[RBA_SAMPLES][KD + 4];
  __shared__ float Gs[KD][PP];
  __shared__ float Cs[RBA_SAMPLES][PP + 1];
  const int tid = threadIdx.x;
  const int kx = K % args.ncx, ky = K / args.ncx;
  for (int idx = tid; idx < RBA_SAMPLES * KD; idx += 256) {
    const int i = idx / KD, e = idx % KD;
    const int64_t s = s0 + i;
    float v = 0.0f;
    if (s < args.nsamples && e < m * m) {
      const TA* a = (const TA*)args.a + s * (int64_t)(args.ncy * m) * lda;
      v = (float)ld(a, (int64_t)(ky * m + e / m) * lda + kx * m + e % m);
    }
    As[i][e] = v;
  }
  const float* G = ra.G32 + (int64_t)K * KD * PP;
  for (int idx = tid; idx < KD * PP; idx += 256) Gs[idx / PP][idx % PP] = G[idx];
  __syncthreads();
  const int w = tid / 64, lane = tid % 64;
  constexpr int NTILE = PP / 16;
  f4 acc[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int kk = 0; kk < KD / 4; ++kk) {
    const float av = As[16 * w + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
      const float bv = Gs[4 * kk + (lane >> 4)][16 * t + (lane & 15)];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) Cs[16 * w + 4 * (lane >> 4) + v][16 * t + (lane & 15)] = acc[t][v];
  __syncthreads();
  if (tid < RBA_SAMPLES) {
    const int64_t s = s0 + tid;
    if (s < args.nsamples) {
      constexpr int P = RMAX * (RMAX + 1) / 2 + 3 * RMAX + 6;
      double v[P];
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = (double)Cs[tid][q];
      double S3[3][3];
      const bool ok = rb_small_solve<RMAX>(v, ra.rK[K], S3);
      const int64_t p = s * Mc + K;
      store_packed(args.S + p * 10, S3);
      if (args.status) args.status[p] = ok ? STOMSFEM_OK : STOMSFEM_ENOTSPD;
    }
  }
}

int rb_pad_p(int rmax) { return ((rb_p(rmax) + 15) / 16) * 16; }
int rb_pad_kd(int m) { return ((m * m + 3) / 4) * 4; }

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
  if (u.m != 8 || ra.KD != 64 || ra.PP != 80) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((u.nsamples + RBA_SAMPLES - 1) / RBA_SAMPLES), (unsigned)(u.ncx * u.ncy));
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL((rb_apply_mfma_kernel<8, 64, 80, float>), grid, dim3(256), 0, st, ra);
  else
    hipLaunchKernelGGL((rb_apply_mfma_kernel<8, 64, 80, double>), grid, dim3(256), 0, st, ra);
  return hipGetLastError();
}

}  // namespace stomsfem
