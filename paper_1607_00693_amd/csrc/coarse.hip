// Batched coarse solve S U = b (Sec. 2.2 eq. upscaleSUF) with the
// Petrov-Galerkin load (eq. stiffness_local_petrov), and the Monte Carlo
// mean / variance of the coarse solution (Sec. 4.1.1).
//
// One workgroup per sample.  The interior coarse nodes in natural order give
// a 9-point band of half-width ncx; the global stiffness rows are assembled
// on the fly from the four upscaled element matrices around each node as
// they enter an LDS window of (ncx+1) x (ncx+1) entries.  FP64 LDL^T with the
// forward substitution fused; the retired columns of L go to a per-workgroup
// slice of the library workspace and are read back once by the backward
// substitution, which is done by one wavefront with a shuffle reduction.
#include "common.h"

namespace stomsfem {

constexpr int COARSE_THREADS = 256;
constexpr int COARSE_NQ = 12;  // largest NQ: B (B+1)/2 <= 3072
constexpr int COARSE_BMAX = 72;

// Workgroup barrier that orders LDS only: a pivot step does not wait for
// its global stores (retired L columns, y_j) to complete.
#define COARSE_SYNC()                                                 \
  do {                                                                \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");   \
    __builtin_amdgcn_s_barrier();                                     \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");   \
  } while (0)

// x mod w for 0 <= x < 2w
__device__ __forceinline__ int wrap(int x, int w) { return x >= w ? x - w : x; }

struct CoarseArgs {
  int32_t ncx, ncy;
  int64_t nsamples;
  const double* S;
  const double* load;
  double* U;
  int32_t* status;
  double* work;  // gridDim.x * nU * (ncx+1) doubles
};

__device__ __forceinline__ double selem(const double* Sk, int i, int j) {
  // packed upper triangle 00,01,02,03,11,12,13,22,23,33
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
  const int base = i == 0 ? 0 : i == 1 ? 4 : i == 2 ? 7 : 9;
  return Sk[base + (j - i)];
}

// NQ = trailing-triangle entries per lane, >= B (B+1) / (2 * 64).
template <int NQ>
__global__ __launch_bounds__(COARSE_THREADS) void coarse_solve_kernel(CoarseArgs args) {
  extern __shared__ double smem[];
  const int ncx = args.ncx, ncy = args.ncy;
  const int nix = ncx - 1, niy = ncy - 1, nU = nix * niy, B = ncx, WN = B + 1;
  double* Wn = smem;        // WN*WN
  double* F = Wn + WN * WN;  // WN (forward-substituted rhs window)
  double* X = F + WN;        // WN (backward substitution window)
  double* Ec = X + WN;       // 4 x ncx x 10: ring of element rows of S (row e in slot e % 4)
  __shared__ int bad;
  __shared__ double colv[COARSE_BMAX];  // pivot column (unscaled), a separate object from the window
  const int tid = threadIdx.x;
  const int Mc = ncx * ncy;
  const double H = 1.0 / ncx;
  double* Lc = args.work + (int64_t)blockIdx.x * nU * WN;  // column j: [d_j, l_{j+1,j}, ..., l_{j+B,j}]
  // entries (io >= ko) of the B x B trailing triangle handled by this lane,
  // the same for every pivot column, packed io | ko << 8 (io = B: unused)
  int tik[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = tid + COARSE_THREADS * q;
    int io = 0;
    while ((io + 1) * (io + 2) / 2 <= t) ++io;
    const bool used = t < B * (B + 1) / 2;
    tik[q] = used ? (io | ((t - io * (io + 1) / 2) << 8)) : B;
  }

  for (int64_t s = blockIdx.x; s < args.nsamples; s += gridDim.x) {
    const double* Ss = args.S + s * (int64_t)Mc * 10;
    double* Us = args.U + s * (int64_t)nU;
    __syncthreads();
    for (int i = tid; i < WN * WN; i += blockDim.x) Wn[i] = 0.0;
    if (tid == 0) bad = 0;
    // Element rows of S go through an LDS ring.  Node row iy uses element rows
    // iy and iy + 1.  Rows 0..3 are loaded here; in the elimination loop
    // (where a barrier follows every inserted row) the first node of node
    // row iy >= 2 loads element row iy + 2 into the slot of row iy - 2, which
    // only node rows up to iy - 2 used; node row iy + 1 needs it nix columns
    // later.
    auto load_erow = [&](int e) {
      if (e < ncy)
        for (int t = tid; t < ncx * 10; t += blockDim.x) Ec[(e % 4) * ncx * 10 + t] = Ss[(int64_t)e * ncx * 10 + t];
    };
    for (int e = 0; e < 4; ++e) load_erow(e);
    __syncthreads();

    // Row r of the coarse system: node (ix, iy) = grid node (px, py); its four
    // elements SW=(px-1,py-1), SE=(px,py-1), NW=(px-1,py), NE=(px,py) see it as
    // local node 2, 3, 1, 0 respectively.
    auto insert_row = [&](int r) {
      const int ix = r % nix, iy = r / nix, px = ix + 1, py = iy + 1;
      if (ix == 0 && iy >= 2 && r >= B) load_erow(iy + 2);
      const double* eS = Ec + ((py - 1) % 4) * ncx * 10;
      const double* eN = Ec + (py % 4) * ncx * 10;
      const double* sSW = eS + (px - 1) * 10;
      const double* sSE = eS + px * 10;
      const double* sNW = eN + (px - 1) * 10;
      const double* sNE = eN + px * 10;
      for (int t = tid; t <= B + 1; t += COARSE_THREADS) {
        if (t > B) {
          double b;
          if (args.load) {
            const double* L = args.load;
            b = (L[((py - 1) * ncx + (px - 1)) * 4 + 2] + L[((py - 1) * ncx + px) * 4 + 3]) +
                (L[(py * ncx + (px - 1)) * 4 + 1] + L[(py * ncx + px) * 4 + 0]);
          } else {
            b = H * H;  // four elements, int_K p^l = H^2/4 each
          }
          F[r % WN] = b;
          continue;
        }
        double v = 0.0;
        if (t == 0) v += (selem(sSW, 2, 2) + selem(sSE, 3, 3)) + (selem(sNW, 1, 1) + selem(sNE, 0, 0));
        if (t == 1 && ix >= 1) v += selem(sSW, 2, 3) + selem(sNW, 1, 0);
        if (t == nix - 1 && iy >= 1 && ix <= nix - 2) v += selem(sSE, 3, 1);
        if (t == nix && iy >= 1) v += selem(sSW, 2, 1) + selem(sSE, 3, 0);
        if (t == nix + 1 && iy >= 1 && ix >= 1) v += selem(sSW, 2, 0);
        if (r - t >= 0) Wn[(r % WN) * WN + ((r - t) % WN)] = v;  // once per row
      }
    };

    for (int r = 0; r < (B < nU ? B : nU); ++r) insert_row(r);
    __syncthreads();
    for (int j = 0; j < nU; ++j) {
      if (j + B < nU) {
        insert_row(j + B);
        COARSE_SYNC();
      }
      const int jj = j % WN;
      const double d = Wn[jj * WN + jj];
      const double inv = 1.0 / d;
      const int cnt = (j + B < nU - 1 ? j + B : nU - 1) - j;
      // column j of L (and the pivot) to the workspace; rhs forward step
      for (int t = tid; t <= cnt; t += COARSE_THREADS) {
        const int rt = wrap(jj + t, WN);
        const double c = Wn[rt * WN + jj];
        const double v = t == 0 ? d : c * inv;
        if (t > 0) colv[t - 1] = c;
        Lc[(int64_t)j * WN + t] = v;
        if (t > 0) F[rt] -= v * F[jj];
      }
      COARSE_SYNC();
      if (tid == 0) {
        if (!(d > 0.0)) bad = 1;
        Us[j] = F[jj];  // y_j, overwritten by x_j below
      }
      // rank-1 update of the trailing triangle, this lane's fixed entries:
      // all reads first, then all writes (distinct addresses), so that the
      // reads are not serialised behind possibly aliasing writes
      {
        double wv[NQ];
        int idx[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int io = tik[q] & 255, ko = tik[q] >> 8;
          idx[q] = wrap(jj + 1 + io, WN) * WN + wrap(jj + 1 + ko, WN);
          wv[q] = io < cnt ? Wn[idx[q]] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int io = tik[q] & 255, ko = tik[q] >> 8;
          if (io < cnt) wv[q] -= colv[io] * inv * colv[ko];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if ((tik[q] & 255) < cnt) Wn[idx[q]] = wv[q];
      }
      COARSE_SYNC();
    }
    // the retired columns and y must be visible to the backward substitution
    __syncthreads();
    // backward substitution x_j = y_j / d_j - sum_{t=1..B} l_{j+t,j} x_{j+t}
    if (tid < 64) {
      for (int t = tid; t < WN; t += 64) X[t] = 0.0;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      for (int j = nU - 1; j >= 0; --j) {
        const double* col = Lc + (int64_t)j * WN;
        double part = 0.0;
        for (int t = 1 + tid; t <= B; t += 64)
          if (j + t < nU) part += col[t] * X[(j + t) % WN];
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
        const double x = Us[j] / col[0] - part;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (tid == 0) {
          X[j % WN] = x;
          Us[j] = x;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
      if (tid == 0 && args.status) args.status[s] = bad ? STOMSFEM_ENOTSPD : STOMSFEM_OK;
    }
  }
}

// qoi_mean[i] = (1/N) sum_s U[s][i]; qoi_var[i] = (1/N) sum_s U^2 - mean^2.
// Fixed summation order over s (bitwise reproducible).
__global__ void qoi_kernel(int64_t N, int nU, const double* U, double* mean, double* var) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nU) return;
  double m1 = 0.0, m2 = 0.0;
  for (int64_t s = 0; s < N; ++s) {
    const double u = U[s * nU + i];
    m1 += u;
    m2 += u * u;
  }
  const double inv = N > 0 ? 1.0 / (double)N : 0.0;
  m1 *= inv;
  m2 *= inv;
  if (mean) mean[i] = m1;
  if (var) var[i] = m2 - m1 * m1;
}

size_t coarse_lds_bytes(int ncx) {
  const int WN = ncx + 1;
  return sizeof(double) * ((size_t)WN * WN + 2 * (size_t)WN + 40 * (size_t)ncx);
}

int64_t coarse_grid(int64_t nsamples) { return nsamples < 4096 ? nsamples : 4096; }

int64_t coarse_work_doubles(int ncx, int ncy, int64_t nsamples) {
  return coarse_grid(nsamples) * (int64_t)(ncx - 1) * (ncy - 1) * (ncx + 1);
}

hipError_t launch_coarse(int ncx, int ncy, int64_t N, const double* S, const double* load, double* U,
                         double* mean, double* var, int32_t* status, double* work, hipStream_t st) {
  const int nU = (ncx - 1) * (ncy - 1);
  if (ncx * (ncx + 1) / 2 > COARSE_THREADS * COARSE_NQ || ncx > COARSE_BMAX) return hipErrorInvalidValue;
  if (N > 0 && nU > 0) {
    CoarseArgs a{ncx, ncy, N, S, load, U, status, work};
    const int need = (ncx * (ncx + 1) / 2 + COARSE_THREADS - 1) / COARSE_THREADS;
    const dim3 grid((unsigned)coarse_grid(N)), block(COARSE_THREADS);
    const size_t lds = coarse_lds_bytes(ncx);
    if (need <= 4)
      hipLaunchKernelGGL(coarse_solve_kernel<4>, grid, block, lds, st, a);
    else
      hipLaunchKernelGGL(coarse_solve_kernel<COARSE_NQ>, grid, block, lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if ((mean || var) && nU > 0) {
    hipLaunchKernelGGL(qoi_kernel, dim3((nU + 255) / 256), dim3(256), 0, st, N, nU, U, mean, var);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace stomsfem
