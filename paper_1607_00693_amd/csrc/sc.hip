// Sparse-grid stochastic collocation with search-and-plug-in dictionaries
// (Sec. 4.1.2, global SC methods, eqs. sparseintegration, SCofflinecost,
// SConlinecost).
//
// Host: the Smolyak combination of nested Clenshaw-Curtis rules.  The
// level-i rule has n_i = 1 (i = 1, the midpoint) or 2^(i-1) + 1 points
// cos(pi j / N), N = n_i - 1, with the classical weights
//   w_j = (c_j / N) (1 - sum_{k=1}^{N/2} b_k cos(2 pi k j / N) / (4k^2 - 1)),
// c_j = 1 at the ends and 2 inside, b_k = 1 at k = N/2 and 2 below (for the
// integral over [-1, 1]; halved here for the uniform probability measure).
// A(L, d) is the sum over multi-indices i >= 1 with max(0, L-d+1) <= |i|-d
// <= L of (-1)^(L+d-|i|) binom(d-1, L+d-|i|) times the tensor rule; the
// rules are nested, so each tensor point is a point of the finest grid of
// the level (digit c <-> cos(pi c / D), D = 2^max(L, 1)) and its weights
// from every term add up.
//
// Device, online stage: sc_apply_kernel, one thread per (point, patch):
// the local point's key (the point's digits at the patch's local variables
// in mixed radix D + 1) is searched by bisection among the patch's sorted
// dictionary keys and the stored S_K is copied out (80 B written per pair).
// sc_quad_*: the weighted sums of U and U^2 over the points, in chunks of
// points (64 unknowns per workgroup, four wavefronts over the chunk's
// points, combined in order), then the chunks in order: a fixed order.
#include "sc.h"

#include <cmath>
#include <functional>
#include <map>

namespace stomsfem {

int64_t sc_term_count(int dim, int level, int64_t cap) {
  // binom(dim + level, level) by the product formula, saturated
  double b = 1.0;
  for (int r = 1; r <= level; ++r) {
    b = b * (double)(dim + r) / (double)r;
    if (b > (double)cap) return cap + 1;
  }
  return (int64_t)std::llround(b);
}

static void cc_rule(int i, int D, std::vector<int32_t>& dig, std::vector<double>& w) {
  dig.clear();
  w.clear();
  if (i == 1) {
    dig.push_back(D / 2);
    w.push_back(1.0);
    return;
  }
  const int N = 1 << (i - 1);
  for (int j = 0; j <= N; ++j) {
    double s = 0.0;
    for (int k = 1; k <= N / 2; ++k) {
      const double bk = (k == N / 2) ? 1.0 : 2.0;
      s += bk * std::cos(2.0 * M_PI * (double)k * (double)j / (double)N) / (4.0 * k * k - 1.0);
    }
    const double cj = (j == 0 || j == N) ? 1.0 : 2.0;
    dig.push_back(j * (D / N));
    w.push_back(0.5 * cj / N * (1.0 - s));
  }
}

static int64_t binom64(int n, int r) {
  int64_t b = 1;
  for (int k = 1; k <= r; ++k) b = b * (n - r + k) / k;
  return b;
}

void sc_smolyak_terms(int dim, int level, const std::function<void(double, const std::vector<int>&)>& term) {
  std::vector<int> idx(dim, 1);
  const int lo_extra = level - dim + 1 > 0 ? level - dim + 1 : 0;
  // depth-first over dimensions distributing the extra levels
  auto rec = [&](auto&& self, int k, int used) -> void {
    if (k == dim) {
      if (used >= lo_extra)
        term(((level - used) % 2 ? -1.0 : 1.0) * (double)binom64(dim - 1, level - used), idx);
      return;
    }
    for (int e = 0; used + e <= level; ++e) {
      idx[k] = 1 + e;
      self(self, k + 1, used + e);
    }
    idx[k] = 1;
  };
  rec(rec, 0, 0);
}

void sc_build_grid(int dim, int level, std::vector<int32_t>& digits, std::vector<double>& weights) {
  const int D = sc_digit_base(level);
  std::vector<std::vector<int32_t>> rd(level + 2);
  std::vector<std::vector<double>> rw(level + 2);
  for (int i = 1; i <= level + 1; ++i) cc_rule(i, D, rd[i], rw[i]);
  std::map<std::vector<int32_t>, double> acc;
  std::vector<int32_t> pt(dim);
  std::vector<int> pos(dim);
  sc_smolyak_terms(dim, level, [&](double c, const std::vector<int>& idx) {
    // tensor product of the rules idx[0..dim-1]
    for (int k = 0; k < dim; ++k) pos[k] = 0;
    while (true) {
      double wt = c;
      for (int k = 0; k < dim; ++k) {
        pt[k] = rd[idx[k]][pos[k]];
        wt *= rw[idx[k]][pos[k]];
      }
      acc[pt] += wt;
      int k = dim - 1;
      while (k >= 0 && ++pos[k] == (int)rd[idx[k]].size()) pos[k--] = 0;
      if (k < 0) break;
    }
  });
  digits.clear();
  weights.clear();
  digits.reserve(acc.size() * (size_t)dim);
  weights.reserve(acc.size());
  for (const auto& kv : acc) {
    digits.insert(digits.end(), kv.first.begin(), kv.first.end());
    weights.push_back(kv.second);
  }
}

__global__ __launch_bounds__(256) void sc_apply_kernel(ScApplyArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.npoints * a.npatch) return;
  const int64_t p = t / a.npatch;
  const int K = (int)(t - p * a.npatch);
  const int k = a.nlv[K];
  const int32_t* dg = a.digits + p * a.nxi;
  int64_t key = 0;
  bool ok = true;
  for (int i = 0; i < k; ++i) {
    const int32_t c = dg[a.lv[K * 4 + i]];
    ok = ok && c >= 0 && c <= a.D;
    key = key * (a.D + 1) + c;
  }
  int64_t lo = a.off[K], hi = a.off[K + 1] - 1, row = -1;
  while (ok && lo <= hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int64_t km = a.keys[mid];
    if (km == key) {
      row = mid;
      break;
    }
    if (km < key) lo = mid + 1;
    else hi = mid - 1;
  }
  double* out = a.S + t * 10;
  if (row >= 0) {
    const double* src = a.table + row * 10;
#pragma unroll
    for (int q = 0; q < 10; ++q) out[q] = src[q];
  } else {
#pragma unroll
    for (int q = 0; q < 10; ++q) out[q] = __builtin_nan("");
  }
  if (a.status) a.status[t] = row >= 0 ? 0 : 1;
}

hipError_t launch_sc_apply(const ScApplyArgs& a, hipStream_t st) {
  const int64_t n = a.npoints * a.npatch;
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sc_apply_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---- sparse-grid interpolation: sgi_apply_kernel ----
// One workgroup = one patch K (blockIdx.y) and 64 samples (one per lane of
// each of its SGI_WAVES wavefronts: 8 up to level 4, 16 at level 5, where
// the bases take twice the LDS), so the patch's table and the
// combination list are read at wave-uniform addresses.  The lanes first
// evaluate, for every local variable d and every level i <= L+1, the
// Lagrange basis of the level-i nodes at the sample's t_d in barycentric
// product form
//   P_j = w_j prod_{e != j} (t - t_e),  l_j = P_j / sum_e P_e,
// w_j = (-1)^j (halved at both ends), the Chebyshev-Lobatto weights (exact on
// a node, no division by zero; level 1: l_0 = 1), into LDS at
// [(d nb + lofs[i] + j) 64 + lane] (lane-interleaved: no bank conflicts);
// wavefront w takes the variables d = w, w + SGI_WAVES, ...  The bases are
// shared by the workgroup's wavefronts, which split the table rows into
// SGI_WAVES consecutive ranges: S_K(t) = sum over the table rows r of
// W_r(t) T_K[r], W_r the sum over the combination entries of node r of
// coef * prod_d B[d][boff_d] (entries are grouped by row, so each table row
// is read once, at a sequential address, and no load address depends on an
// earlier load).  The wavefronts' partial sums are added in wavefront order
// through LDS (over the bases, after a barrier), and the first wavefront
// stores.  Lanes with a local variable outside [lo, hi] (or NaN) are listed
// for the plain path instead.  Every global store (and the list's atomic)
// comes after the loop, so the wave-uniform loads of the loop are not
// clobbered and go through the scalar cache.
template <int SGI_WAVES, int NE>
__global__ __launch_bounds__(64 * SGI_WAVES) void sgi_apply_kernel(SgiApplyArgs a) {
  extern __shared__ double sgi_lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int K = blockIdx.y;
  const int64_t s = (int64_t)blockIdx.x * 64 + lane;
  const bool valid = s < a.nsamples;
  const int k = a.nlv[K];
  double* B = sgi_lds + lane;  // B[e * 64] = basis value e of this lane's sample
  bool inside = valid;
  for (int d = 0; d < k; ++d) {
    const double x = valid ? a.xi[s * a.nxi + a.lv[K * 4 + d]] : 0.0;
    inside = inside && (x >= a.lo && x <= a.hi);
    if (d % SGI_WAVES != wave) continue;
    const double t = 2.0 * (x - a.lo) / (a.hi - a.lo) - 1.0;
    double* Bd = B + d * a.nb * 64;
    Bd[0] = 1.0;  // level 1
    for (int i = 2; i <= a.level + 1; ++i) {
      const int n = (1 << (i - 1)) + 1, o = a.lofs[i];
      double sum = 0.0;
      for (int j = 0; j < n; ++j) {
        double P = (j & 1) ? -1.0 : 1.0;
        if (j == 0 || j == n - 1) P *= 0.5;
        for (int e = 0; e < n; ++e)
          if (e != j) P *= t - a.nodes[o + e];
        Bd[(o + j) * 64] = P;
        sum += P;
      }
      const double r = 1.0 / sum;
      for (int j = 0; j < n; ++j) Bd[(o + j) * 64] *= r;
    }
  }
  __syncthreads();
  const int64_t p = s * a.npatch + K;
  double acc[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) acc[q] = 0.0;
  const double* T = a.table + a.off[K] * NE;
  const int32_t* rs = a.cb_rows + a.rofs[k];  // entries of row r: rs[r] .. rs[r+1]-1
  const int nr = a.rofs[k + 1] - a.rofs[k] - 1;
  const int r0 = (int)((int64_t)nr * wave / SGI_WAVES), r1 = (int)((int64_t)nr * (wave + 1) / SGI_WAVES);
  int c = rs[r0];
  for (int r = r0; r < r1; ++r) {
    const int c1 = rs[r + 1];
    double wr = 0.0;
    // SGI_BATCH entries at a time, so that their LDS reads are in flight
    // together; the entry arrays carry SGI_BATCH - 1 padding entries, and
    // entries past the row's end count as zero (the sum keeps its order)
    for (; c < c1; c += SGI_BATCH) {
      double w[SGI_BATCH];
      uint32_t bo[SGI_BATCH];
#pragma unroll
      for (int u = 0; u < SGI_BATCH; ++u) {
        w[u] = c + u < c1 ? a.cb_coef[c + u] : 0.0;
        bo[u] = a.cb_boff[c + u];
      }
      for (int d = 0; d < k; ++d)
#pragma unroll
        for (int u = 0; u < SGI_BATCH; ++u) w[u] *= B[(d * a.nb + (int)((bo[u] >> (8 * d)) & 255u)) * 64];
#pragma unroll
      for (int u = 0; u < SGI_BATCH; ++u) wr += w[u];
    }
    c = c1;
    const double* Tr = T + (int64_t)r * NE;
#pragma unroll
    for (int q = 0; q < NE; ++q) acc[q] += wr * Tr[q];
  }
  // partial sums of wavefronts 1.. into LDS (the bases are no longer read)
  __syncthreads();
  double* red = sgi_lds + lane;  // red[((w - 1) * NE + q) * 64]
  if (wave > 0) {
#pragma unroll
    for (int q = 0; q < NE; ++q) red[((wave - 1) * NE + q) * 64] = acc[q];
  }
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int w = 1; w < SGI_WAVES; ++w)
#pragma unroll
    for (int q = 0; q < NE; ++q) acc[q] += red[((w - 1) * NE + q) * 64];
  if (valid && inside) {
    double* So = a.S + p * NE;
#pragma unroll
    for (int q = 0; q < NE; ++q) So[q] = acc[q];
    if (a.status) a.status[p] = 0;
  } else if (valid) {
    const unsigned long long slot = atomicAdd(a.list_count, 1ull);
    a.list[slot] = p;
  }
}

static int sgi_waves(int level) { return level >= 5 ? 16 : 8; }

size_t sgi_lds_bytes(int kmax, int nb, int level, int ne) {
  const size_t bases = (size_t)64 * (kmax > 0 ? kmax : 1) * nb * sizeof(double);
  const size_t red = (size_t)64 * (sgi_waves(level) - 1) * ne * sizeof(double);
  return bases > red ? bases : red;
}

template <int NW, int NE>
static hipError_t launch_sgi(const SgiApplyArgs& a, hipStream_t st) {
  const size_t lds = sgi_lds_bytes(a.kmax, a.nb, a.level, NE);
  hipError_t e = hipFuncSetAttribute((const void*)sgi_apply_kernel<NW, NE>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((a.nsamples + 63) / 64), (unsigned)a.npatch);
  hipLaunchKernelGGL((sgi_apply_kernel<NW, NE>), grid, dim3(64 * NW), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_sgi_apply(const SgiApplyArgs& a, hipStream_t st) {
  if (a.nsamples == 0) return hipSuccess;
  const bool w16 = sgi_waves(a.level) == 16;
  if (a.ne == 16) return w16 ? launch_sgi<16, 16>(a, st) : launch_sgi<8, 16>(a, st);
  if (a.ne != 0 && a.ne != 10) return hipErrorInvalidValue;
  return w16 ? launch_sgi<16, 10>(a, st) : launch_sgi<8, 10>(a, st);
}

static int64_t quad_chunk(int64_t npoints) {
  int64_t ch = 256;
  while ((npoints + ch - 1) / ch > 65535) ch *= 2;
  return ch;
}

int64_t sc_quad_work_doubles(int64_t npoints, int nu) {
  const int64_t ch = quad_chunk(npoints);
  return ((npoints + ch - 1) / ch) * (int64_t)nu * 2;
}

__global__ __launch_bounds__(256) void sc_quad_partial_kernel(const double* __restrict__ U,
                                                              const double* __restrict__ w, int64_t npoints, int nu,
                                                              int64_t ch, double* __restrict__ work) {
  __shared__ double red[4][64][2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int64_t c = blockIdx.y;
  const int64_t p0 = c * ch, p1 = p0 + ch < npoints ? p0 + ch : npoints;
  double s1 = 0.0, s2 = 0.0;
  if (i < nu) {
    for (int64_t p = p0 + wv; p < p1; p += 4) {
      const double u = U[p * nu + i], wp = w[p];
      s1 += wp * u;
      s2 += wp * u * u;
    }
  }
  red[wv][lane][0] = s1;
  red[wv][lane][1] = s2;
  __syncthreads();
  if (wv == 0 && i < nu) {
    double t1 = 0.0, t2 = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      t1 += red[v][lane][0];
      t2 += red[v][lane][1];
    }
    work[(c * nu + i) * 2] = t1;
    work[(c * nu + i) * 2 + 1] = t2;
  }
}

__global__ __launch_bounds__(64) void sc_quad_final_kernel(const double* __restrict__ work, int64_t nchunks, int nu,
                                                           double* __restrict__ mean, double* __restrict__ var) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= nu) return;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t c = 0; c < nchunks; ++c) {
    s1 += work[(c * nu + i) * 2];
    s2 += work[(c * nu + i) * 2 + 1];
  }
  if (mean) mean[i] = s1;
  if (var) var[i] = s2 - s1 * s1;
}

hipError_t launch_sc_quadrature(const double* U, const double* w, int64_t npoints, int nu, double* mean, double* var,
                                double* work, hipStream_t st) {
  const int64_t ch = quad_chunk(npoints);
  const int64_t nchunks = (npoints + ch - 1) / ch;
  const unsigned bx = (unsigned)((nu + 63) / 64);
  hipLaunchKernelGGL(sc_quad_partial_kernel, dim3(bx, (unsigned)nchunks), dim3(256), 0, st, U, w, npoints, nu, ch,
                     work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sc_quad_final_kernel, dim3(bx), dim3(64), 0, st, work, nchunks, nu, mean, var);
  return hipGetLastError();
}

}  // namespace stomsfem
