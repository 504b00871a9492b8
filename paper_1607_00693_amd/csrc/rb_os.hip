// Reduced basis on oversampled patches (Sec. 3.2 with the oversampled
// Petrov-Galerkin MsFEM of Sec. 2.2; the high-contrast example of Sec. 5.2
// combines them).
//
// The cell problems of element K are posed on its oversampled patch (side
// Mp = m + 2o, moved inside the domain where it would stick out) with the
// bilinear data of the patch corners.  Offline, the patch blocks of the
// training samples are gathered (rb_os_embed_kernel) and reduced exactly as
// plain patches (rb.hip: means phibar^l, KL modes zeta_q in the energy of the
// training-mean coefficient, element table G).  Online, per pair, the reduced
// patch solutions are
//     psi^l = phibar^l + sum_q c^l_q zeta_q,  A c^l = -Fh_l,  l = 0..2,
//     psi^3 = 1 - sum_l psi^l,
// and the element stiffness follows the oversampled recombination: Psi[k][j]
// = psi^j at K's corners x_k, the trial functions phi^i = sum_j C[i][j] psi^j
// with C = Psi^{-T} (phi^i(x_k) = delta_ik), and
//     S16[i][l'] = int_K a grad phi^i . grad p^l' = (Psi^{-T} T)[i][l'],
//     T[j][l'] = int_K a grad psi^j . grad p^l'
//              = U[j][l'] + sum_q c^j_q U[3+q][l'],   T[3][.] = -sum_j T[j][.]
// where U[f][l'] = sum_{e in K} a_e f_e . K_ref p_e^l' for the fields
// f = phibar^0..2, zeta_0..7, with p^l' the bilinear functions of K.  Every
// linear quantity (A, Fh, U) is a linear function of the patch's coefficient
// values; the table GO holds their per-element coefficients (rb.h), so the
// online stage is one pass over the patch, an r x r LDL^T solve, and the
// 4 x 4 recombination.
#include "rb.h"
#include "rb_os_dev.h"

namespace stomsfem {

namespace {

// Bilinear function of corner l of an m x m element at its local node (u, v),
// corners counter-clockwise from the lower left.
__device__ inline double rbo_bil(int l, int u, int v, int m) {
  const double x = (double)u / m, y = (double)v / m;
  return l == 0 ? (1.0 - x) * (1.0 - y) : l == 1 ? x * (1.0 - y) : l == 2 ? x * y : (1.0 - x) * y;
}

__device__ constexpr int RBO_DX[4] = {0, 1, 1, 0};
__device__ constexpr int RBO_DY[4] = {0, 0, 1, 1};

}  // namespace

// Patch blocks of every (sample, element): out[s][ky*Mp + i][kx*Mp + j] =
// a[s][y0(ky) + i][x0(kx) + j] (FP64), the layout of a batch whose elements
// are the patches.
template <typename TA>
__global__ __launch_bounds__(256) void rb_os_embed_kernel(const TA* a, int64_t total, int ncx, int ncy, int m,
                                                          int o, double* out) {
  const int Mp = m + 2 * o, nfx = ncx * m, nfy = ncy * m, W = ncx * Mp;
  const int64_t per_s = (int64_t)ncy * Mp * W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / per_s;
    const int64_t r = i - s * per_s;
    const int Y = (int)(r / W), X = (int)(r % W);
    const int ky = Y / Mp, iy = Y % Mp, kx = X / Mp, ix = X % Mp;
    const int x0 = rbo_origin(kx, m, o, nfx), y0 = rbo_origin(ky, m, o, nfy);
    out[i] = ld(a, s * nfy * nfx + (int64_t)(y0 + iy) * nfx + x0 + ix);
  }
}

// Online tables of patch K (one workgroup per patch).
__global__ __launch_bounds__(256) void rb_os_tables_kernel(RbOsArgs t) {
  const int K = blockIdx.x;
  const int kx = K % t.ncx, ky = K / t.ncx, m = t.m, Mp = t.Mp, n = Mp - 1, nI = n * n, rmax = t.rmax;
  const int cx = kx * m - rbo_origin(kx, m, t.o, t.ncx * m);
  const int cy = ky * m - rbo_origin(ky, m, t.o, t.ncy * m);
  const double* Zk = t.Z + (int64_t)K * nI * rmax;
  const double* pb = t.phibar + (int64_t)K * 3 * nI;
  // field f at patch node (px, py): phibar^f (with the boundary data of the
  // patch corners) for f < 3, zeta_{f-3} (zero on the boundary) otherwise
  auto field = [&](int f, int px, int py) -> double {
    const bool inner = px > 0 && px < Mp && py > 0 && py < Mp;
    if (!inner) return f < 3 ? pcorner(f, px, py, Mp) : 0.0;
    const int id = (py - 1) * n + (px - 1);
    return f < 3 ? pb[f * nI + id] : Zk[id * rmax + (f - 3)];
  };
  double* GO = t.GO + (int64_t)K * t.KDo * RBO_PO;
  float* GO32 = t.GO32 + (int64_t)K * t.KDo * RBO_PO;
  const double* G = t.G64 + (int64_t)K * t.KD * t.PP;
  for (int idx = threadIdx.x; idx < t.KDo * RBO_PO; idx += blockDim.x) {
    const int e = idx / RBO_PO, c = idx % RBO_PO;
    double val = 0.0;
    if (e < Mp * Mp) {
      if (c < RBO_H) {
        val = G[(int64_t)e * t.PP + c];
      } else if (c < RBO_H + 4 * RBO_NF) {
        const int ex = e % Mp, ey = e / Mp, ix = ex - cx, iy = ey - cy;
        if (ix >= 0 && ix < m && iy >= 0 && iy < m) {
          const int f = (c - RBO_H) / 4, lp = (c - RBO_H) % 4;
          for (int al = 0; al < 4; ++al) {
            const double fv = field(f, ex + RBO_DX[al], ey + RBO_DY[al]);
            for (int be = 0; be < 4; ++be) val += fv * kref(al, be) * rbo_bil(lp, ix + RBO_DX[be], iy + RBO_DY[be], m);
          }
        }
      }
    }
    GO[idx] = val;
    GO32[idx] = (float)val;
  }
  for (int idx = threadIdx.x; idx < 4 * RBO_NF; idx += blockDim.x) {
    const int k = idx / RBO_NF, f = idx % RBO_NF;
    t.Pc[(int64_t)K * 4 * RBO_NF + idx] = field(f, cx + m * RBO_DX[k], cy + m * RBO_DY[k]);
  }
}

// FP64 online stage.  One lane per pair; a wavefront holds 64 samples of one
// patch, so that the patch's table rows are wavefront-uniform.
template <typename TA>
__global__ __launch_bounds__(256) void rb_os_apply_f64_kernel(RbOsArgs t, UpArgs up, int64_t nsb) {
  constexpr int RMAX = 8, NV = RBO_H;
  const int Mc = t.ncx * t.ncy;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int K = __builtin_amdgcn_readfirstlane((int)(w / nsb));
  if (K >= Mc) return;
  const int64_t s = (w - (int64_t)K * nsb) * 64 + (threadIdx.x & 63);
  if (s >= up.nsamples) return;
  const int m = t.m, Mp = t.Mp, kx = K % t.ncx, ky = K / t.ncx;
  const int nfx = t.ncx * m, nfy = t.ncy * m;
  const int x0 = rbo_origin(kx, m, t.o, nfx), y0 = rbo_origin(ky, m, t.o, nfy);
  const TA* a = (const TA*)up.a + s * nfy * nfx + (int64_t)y0 * nfx + x0;
  const double* GO = t.GO + (int64_t)K * t.KDo * RBO_PO;
  // pass 1: A and Fh of the reduced patch system over the whole patch
  double v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = 0.0;
  for (int ey = 0; ey < Mp; ++ey)
    for (int ex = 0; ex < Mp; ++ex) {
      const double ae = ld(a, (int64_t)ey * nfx + ex);
      const double* g = GO + (int64_t)(ey * Mp + ex) * RBO_PO;
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] += ae * g[q];
    }
  double c[3][RMAX];
  const bool ok = rbo_coeffs<RMAX>(v, t.rK[K], c);
  // pass 2: U over the elements of K
  const int cx = kx * m - x0, cy = ky * m - y0;
  double Uf[4 * RBO_NF];  // U[f][l'] at 4 f + l'
#pragma unroll
  for (int q = 0; q < 4 * RBO_NF; ++q) Uf[q] = 0.0;
  for (int iy = 0; iy < m; ++iy)
    for (int ix = 0; ix < m; ++ix) {
      const int ex = cx + ix, ey = cy + iy;
      const double ae = ld(a, (int64_t)ey * nfx + ex);
      const double* g = GO + (int64_t)(ey * Mp + ex) * RBO_PO + RBO_H;
#pragma unroll
      for (int q = 0; q < 4 * RBO_NF; ++q) Uf[q] += ae * g[q];
    }
  double S[4][4];
  const bool nonsing = rbo_recombine<RMAX>(c, Uf, t.Pc + (int64_t)K * 4 * RBO_NF, S);
  double* out = up.S + (s * Mc + K) * 16;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int lp = 0; lp < 4; ++lp) out[4 * i + lp] = S[i][lp];
  if (up.status) up.status[s * Mc + K] = (ok && nonsing) ? STOMSFEM_OK : STOMSFEM_ENOTSPD;
}

hipError_t launch_rb_os_embed(const void* a, int a_dtype, int64_t nsamples, int ncx, int ncy, int m, int o,
                              double* out, hipStream_t st) {
  const int Mp = m + 2 * o;
  const int64_t total = nsamples * ncy * Mp * (int64_t)ncx * Mp;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(rb_os_embed_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, (const float*)a, total,
                       ncx, ncy, m, o, out);
  else
    hipLaunchKernelGGL(rb_os_embed_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, (const double*)a,
                       total, ncx, ncy, m, o, out);
  return hipGetLastError();
}

hipError_t launch_rb_os_tables(const RbOsArgs& t, hipStream_t st) {
  if (t.rmax != 8 || rb_na(t.rmax) + 3 * t.rmax != RBO_H || t.KDo < t.Mp * t.Mp || t.KD < t.Mp * t.Mp)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(rb_os_tables_kernel, dim3((unsigned)(t.ncx * t.ncy)), dim3(256), 0, st, t);
  return hipGetLastError();
}

hipError_t launch_rb_os_apply(const RbOsArgs& t, const UpArgs& up, int a_dtype, hipStream_t st) {
  if (up.nsamples == 0) return hipSuccess;
  if (t.rmax != 8 || up.m != t.m || up.ncx != t.ncx || up.ncy != t.ncy) return hipErrorInvalidValue;
  const int64_t nsb = (up.nsamples + 63) / 64, waves = nsb * t.ncx * t.ncy, blocks = (waves + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(rb_os_apply_f64_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, t, up, nsb);
  else
    hipLaunchKernelGGL(rb_os_apply_f64_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, t, up, nsb);
  return hipGetLastError();
}

}  // namespace stomsfem
