// Random interpolation of the upscaled stiffness (Sec. 3.1).
//
// Offline (Algorithm 1), per patch K with k local variables: the nn^k tensor
// nodes of the Chebyshev-Gauss-Lobatto points of the box [lo, hi]; the plain
// path gives S_K at every node.  The kernels here generate the node random
// vectors (ri_nodes_kernel) and regenerate the coefficient blocks of listed
// (sample, patch) pairs from their random vectors (regen_blocks_kernel); the
// host runs the ordinary upscaling kernels on those blocks.
//
// Online (Algorithm 2), ri_apply_kernel: one lane per (sample, patch), every
// lane of a workgroup on the same patch, so the table is read at wave-uniform
// addresses (scalar loads, shared through the caches).  The 1-D basis values
// of variable i are l_d(x) = P_d / sum_e P_e with
//   P_d = w_d prod_{e != d} (x - t_e),  w_d = (-1)^d (1/2 at d = 0, nn-1),
// the Chebyshev-Lobatto barycentric weights (Berrut & Trefethen 2004) with
// the node polynomial multiplied through, so an evaluation exactly on a node
// needs no special case and constants are reproduced exactly.  S_K is then
// sum_c prod_i l_{d_i}(x_i) T_K[c]: the two fastest variables are unrolled
// (only the fastest above five nodes), the others are runtime loops.
#include "ri.h"

namespace stomsfem {

__device__ __forceinline__ double cgl_node(int d, int nn, double lo, double hi) {
  return lo + (cos(M_PI * (double)d / (double)(nn - 1)) + 1.0) * 0.5 * (hi - lo);
}

__global__ __launch_bounds__(256) void ri_nodes_kernel(RiNodeArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.count) return;
  const int64_t row = a.start + i;
  // patch owning the row: off is sorted, off[0] = 0, off[npatch] = rows
  int lo = 0, hi = a.npatch - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.off[mid] <= row) lo = mid;
    else hi = mid - 1;
  }
  const int K = lo;
  double* x = a.xi_out + i * a.nxi;
  for (int j = 0; j < a.nxi; ++j) x[j] = 0.0;
  const int k = a.nlv[K];
  int64_t c = row - a.off[K];
  for (int v = k - 1; v >= 0; --v) {  // last variable = fastest digit
    const int d = (int)(c % a.nn);
    c /= a.nn;
    x[a.lv[K * RI_KMAX + v]] = cgl_node(d, a.nn, a.lo, a.hi);
  }
  a.pairs_out[i] = i * a.npatch + K;
}

__global__ __launch_bounds__(256) void regen_blocks_kernel(RegenArgs a) {
  const int64_t mm = (int64_t)a.m * a.m;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.count * mm) return;
  const int64_t i = t / mm;
  const int e = (int)(t - i * mm);
  const int64_t npatch = (int64_t)a.ncx * a.ncy;
  const int64_t p = a.pairs[i];
  const int64_t s = p / npatch;
  const int K = (int)(p - s * npatch);
  const int kx = K % a.ncx, ky = K / a.ncx;
  const int ex = e % a.m, ey = e / a.m;
  if (a.fmap) {
    const int32_t f = a.fmap[(int64_t)(ky * a.m + ey) * ((int64_t)a.ncx * a.m) + kx * a.m + ex];
    a.out[t] = (unsigned)f < (unsigned)a.nxi ? feature_theta(a.xi[s * a.nxi + f], a.decades) : 1.0;
    return;
  }
  const double h = 1.0 / ((double)a.ncx * a.m);
  a.out[t] = bump_coef((kx * a.m + ex + 0.5) * h, (ky * a.m + ey + 0.5) * h, a.xi + s * a.nxi, a.bp);
}

__global__ __launch_bounds__(256) void scatter_pairs_kernel(const int64_t* __restrict__ pairs, int64_t count,
                                                            const double* __restrict__ Sc,
                                                            const int32_t* __restrict__ stc, double* __restrict__ S,
                                                            int32_t* __restrict__ status, int32_t code,
                                                            int ne) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const int64_t p = pairs[i];
  for (int q = 0; q < ne; ++q) S[p * ne + q] = Sc[i * ne + q];
  if (status) status[p] = stc[i] != 0 ? stc[i] : code;
}

__global__ void clear_u64_kernel(unsigned long long* p) {
  if (threadIdx.x == 0) *p = 0ull;
}

// The table is read-only during the online kernel: reading it through the
// constant address space lets wave-uniform addresses use scalar loads.
typedef __attribute__((address_space(4))) const double table_t;

// Drop the first entry of v (v[q] <- v[q+1]): lets a runtime loop walk an
// array held in registers without dynamic indexing.
template <int NN>
__device__ __forceinline__ void shift_down(double (&v)[NN]) {
#pragma unroll
  for (int q = 0; q + 1 < NN; ++q) v[q] = v[q + 1];
}

// Basis values c[d] = l_d(x) on the NN Lobatto nodes of [lo, hi].
template <int NN>
__device__ __forceinline__ void lobatto_basis(double x, double lo, double hi, double (&c)[NN]) {
  double dx[NN];
#pragma unroll
  for (int d = 0; d < NN; ++d) dx[d] = x - cgl_node(d, NN, lo, hi);
  double pre[NN];
  pre[0] = 1.0;
#pragma unroll
  for (int d = 1; d < NN; ++d) pre[d] = pre[d - 1] * dx[d - 1];
  double suf = 1.0, sum = 0.0;
#pragma unroll
  for (int d = NN - 1; d >= 0; --d) {
    const double w = ((d & 1) ? -1.0 : 1.0) * ((d == 0 || d == NN - 1) ? 0.5 : 1.0);
    c[d] = w * pre[d] * suf;
    sum += c[d];
    suf *= dx[d];
  }
  const double inv = 1.0 / sum;
#pragma unroll
  for (int d = 0; d < NN; ++d) c[d] *= inv;
}

// acc += w * sum_{d2, d3} c2[d2] c3[d3] T[(d2 NN + d3) NE + e]  (two fastest
// variables; K2 = how many of them are present, 0..2; NE entries per row).
template <int NN, int K2, int NE>
__device__ __forceinline__ void inner_sum(const table_t* T, double w, const double (&c2)[NN],
                                          const double (&c3)[NN], double (&acc)[NE]) {
  if constexpr (K2 == 0) {
#pragma unroll
    for (int e = 0; e < NE; ++e) acc[e] = fma(w, T[e], acc[e]);
  } else if constexpr (K2 == 1) {
#pragma unroll
    for (int d = 0; d < NN; ++d) {
      const double wd = w * c3[d];
#pragma unroll
      for (int e = 0; e < NE; ++e) acc[e] = fma(wd, T[d * NE + e], acc[e]);
    }
  } else {
#pragma unroll
    for (int d2 = 0; d2 < NN; ++d2) {
      const double w2 = w * c2[d2];
#pragma unroll
      for (int d3 = 0; d3 < NN; ++d3) {
        const double wd = w2 * c3[d3];
#pragma unroll
        for (int e = 0; e < NE; ++e) acc[e] = fma(wd, T[(d2 * NN + d3) * NE + e], acc[e]);
      }
    }
  }
}

// Sum over the two fastest variables for NN > 5: only the fastest is
// unrolled (NN x NE table values per block instead of NN^2 x NE, which
// would exceed the scalar registers and serialise the scalar loads).
template <int NN, int NE>
__device__ __forceinline__ void inner_sum_rows(const table_t* T, double w, const double (&c2)[NN],
                                               const double (&c3)[NN], double (&acc)[NE]) {
  double c2r[NN];
#pragma unroll
  for (int q = 0; q < NN; ++q) c2r[q] = c2[q];
#pragma unroll 1
  for (int d2 = 0; d2 < NN; ++d2) {
    inner_sum<NN, 1, NE>(T + (int64_t)d2 * NN * NE, w * c2r[0], c2, c3, acc);
    shift_down<NN>(c2r);
  }
}

// two fastest variables: unrolled (NN <= 5) or a loop over the second
template <int NN, int NE>
__device__ __forceinline__ void inner_sum2(const table_t* T, double w, const double (&c2)[NN],
                                           const double (&c3)[NN], double (&acc)[NE]) {
  if constexpr (NN > 5)  // measured: at five nodes the full unroll is 4% faster
    inner_sum_rows<NN, NE>(T, w, c2, c3, acc);
  else
    inner_sum<NN, 2, NE>(T, w, c2, c3, acc);
}

template <int NN, int KV, int NE>
__device__ __forceinline__ void ri_eval(const table_t* T, const double (&x)[RI_KMAX], double lo,
                                        double hi, double (&acc)[NE]) {
  double c0[NN], c1[NN], c2[NN], c3[NN];
  // variables are consumed from the fastest: the last one pairs with c3
  if constexpr (KV >= 1) lobatto_basis<NN>(x[KV - 1], lo, hi, c3);
  if constexpr (KV >= 2) lobatto_basis<NN>(x[KV - 2], lo, hi, c2);
  if constexpr (KV >= 3) lobatto_basis<NN>(x[KV - 3], lo, hi, c1);
  if constexpr (KV >= 4) lobatto_basis<NN>(x[KV - 4], lo, hi, c0);
  constexpr int K2 = KV < 2 ? KV : 2;
  constexpr int inner = K2 == 0 ? 1 : (K2 == 1 ? NN : NN * NN);
  if constexpr (KV == 2) {
    inner_sum2<NN, NE>(T, 1.0, c2, c3, acc);
  } else if constexpr (KV < 2) {
    inner_sum<NN, K2, NE>(T, 1.0, c2, c3, acc);
  } else if constexpr (KV == 3) {
#pragma unroll 1
    for (int d1 = 0; d1 < NN; ++d1) {
      inner_sum2<NN, NE>(T + (int64_t)d1 * inner * NE, c1[0], c2, c3, acc);
      shift_down<NN>(c1);
    }
  } else {
#pragma unroll 1
    for (int d0 = 0; d0 < NN; ++d0) {
      double c1r[NN];
#pragma unroll
      for (int q = 0; q < NN; ++q) c1r[q] = c1[q];
#pragma unroll 1
      for (int d1 = 0; d1 < NN; ++d1) {
        inner_sum2<NN, NE>(T + (int64_t)(d0 * NN + d1) * inner * NE, c0[0] * c1r[0], c2, c3, acc);
        shift_down<NN>(c1r);
      }
      shift_down<NN>(c0);
    }
  }
}

// Grid: ceil(nsamples / 256) x npatch workgroups in one dimension, remapped
// so that all workgroups of one patch run on the same XCD (workgroups are
// dealt to the 8 XCDs round-robin), which keeps each table in one L2.
template <int NN, int NE>
__global__ __launch_bounds__(256) void ri_apply_kernel(RiApplyArgs a, int64_t nblk_s, int64_t nwork) {
  const int64_t b = blockIdx.x;
  const int64_t per_xcd = (int64_t)gridDim.x / 8;
  const int64_t w = (b % 8) * per_xcd + b / 8;
  if (w >= nwork) return;
  const int K = (int)(w / nblk_s);
  const int64_t s = (w - (int64_t)K * nblk_s) * 256 + threadIdx.x;
  if (s >= a.nsamples) return;
  const int k = a.nlv[K];
  double x[RI_KMAX] = {0.0, 0.0, 0.0, 0.0};
  bool inside = true;
#pragma unroll
  for (int i = 0; i < RI_KMAX; ++i)
    if (i < k) {
      x[i] = a.xi[s * a.nxi + a.lv[K * RI_KMAX + i]];
      inside = inside && (x[i] >= a.lo && x[i] <= a.hi);
    }
  const int64_t p = s * a.npatch + K;
  if (!inside) {
    const unsigned long long slot = atomicAdd(a.list_count, 1ull);
    a.list[slot] = p;
    return;  // S and status are written by the plain solve
  }
  const table_t* T = (const table_t*)(a.table + a.off[K] * NE);
  double acc[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) acc[e] = 0.0;
  switch (k) {
    case 0: ri_eval<NN, 0, NE>(T, x, a.lo, a.hi, acc); break;
    case 1: ri_eval<NN, 1, NE>(T, x, a.lo, a.hi, acc); break;
    case 2: ri_eval<NN, 2, NE>(T, x, a.lo, a.hi, acc); break;
    case 3: ri_eval<NN, 3, NE>(T, x, a.lo, a.hi, acc); break;
    default: ri_eval<NN, 4, NE>(T, x, a.lo, a.hi, acc); break;
  }
  double* So = a.S + p * NE;
#pragma unroll
  for (int e = 0; e < NE; ++e) So[e] = acc[e];
  if (a.status) a.status[p] = 0;
}

hipError_t launch_ri_nodes(const RiNodeArgs& a, hipStream_t st) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(ri_nodes_kernel, dim3((unsigned)((a.count + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_regen_blocks(const RegenArgs& a, hipStream_t st) {
  if (a.count <= 0) return hipSuccess;
  const int64_t n = a.count * a.m * a.m;
  hipLaunchKernelGGL(regen_blocks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_scatter_pairs(const int64_t* pairs, int64_t count, const double* Sc, const int32_t* stc, double* S,
                                int32_t* status, int32_t code, hipStream_t st, int ne) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_pairs_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, pairs, count, Sc,
                     stc, S, status, code, ne);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t st) {
  hipLaunchKernelGGL(clear_u64_kernel, dim3(1), dim3(64), 0, st, p);
  return hipGetLastError();
}

template <int NN>
static hipError_t launch_apply_nn(const RiApplyArgs& a, hipStream_t st) {
  const int64_t nblk_s = (a.nsamples + 255) / 256;
  const int64_t nwork = nblk_s * a.npatch;
  const int64_t grid = (nwork + 7) / 8 * 8;
  if (a.ne == 16)
    hipLaunchKernelGGL((ri_apply_kernel<NN, 16>), dim3((unsigned)grid), dim3(256), 0, st, a, nblk_s, nwork);
  else if (a.ne == 0 || a.ne == 10)
    hipLaunchKernelGGL((ri_apply_kernel<NN, 10>), dim3((unsigned)grid), dim3(256), 0, st, a, nblk_s, nwork);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_ri_apply(const RiApplyArgs& a, hipStream_t st) {
  if (a.nsamples <= 0) return hipSuccess;
  switch (a.nn) {
    case 2: return launch_apply_nn<2>(a, st);
    case 3: return launch_apply_nn<3>(a, st);
    case 4: return launch_apply_nn<4>(a, st);
    case 5: return launch_apply_nn<5>(a, st);
    case 6: return launch_apply_nn<6>(a, st);
    case 7: return launch_apply_nn<7>(a, st);
    case 8: return launch_apply_nn<8>(a, st);
    case 9: return launch_apply_nn<9>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace stomsfem
