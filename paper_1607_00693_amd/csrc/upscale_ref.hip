// Reference local upscaling kernel: one workgroup per (coarse element,
// sample) pair, any m.  Same mathematics as the tuned kernels (Schur
// complement onto the boundary through a sliding LDL^T window, Sec. 2.2
// eqs. MsFEB and stiffness_local), written for clarity: the coefficient block
// and the (m+1) x (m+1) band window live in LDS and every pivot step is a
// workgroup-wide rank-1 update between two barriers.  It exists to
// cross-check the register-blocked kernels and to serve unusual m, and it is
// the kernel of the oscillatory boundary data: on each edge of K the 1-D
// discrete harmonic profile of the edge-adjacent fine elements,
//   u(t) = sum_{s >= t} 1/a_s / sum_s 1/a_s   (1 at t = 0, 0 at t = m),
// taken by the corner at t = 0 as u and by the corner at t = m as 1 - u
// (edges: bottom from corner 0 to 1, right from 1 to 2, top from 3 to 2,
// left from 0 to 3).  The three data sets still sum with the fourth to 1 on
// the boundary, so S 1 = 0 and the fourth row follows as before.
#include "common.h"

namespace stomsfem {

constexpr int REF_THREADS = 256;

template <typename T>
__global__ __launch_bounds__(REF_THREADS) void upscale_ref_kernel(UpArgs args) {
  extern __shared__ double smem[];
  const int m = args.m, n = m - 1, NI = n * n, B = m, WN = B + 1;
  double* A = smem;                 // m*m coefficient block
  double* Wn = A + m * m;           // WN*WN window, (r, c) at [r%WN][c%WN]
  double* F = Wn + WN * WN;         // WN*3
  double* Gp = F + WN * 3;          // 4 x (m+1): oscillatory profiles u_e(t) per edge
  __shared__ double sbb_part[REF_THREADS / 64][6];
  const bool osc = args.bc == STOMSFEM_BC_OSCILLATORY;
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int Mc = args.ncx * args.ncy;
  const int64_t lda = (int64_t)args.ncx * m;

  for (int64_t p = blockIdx.x; p < args.npairs; p += gridDim.x) {
    const int64_t s = p / Mc;
    const int K = (int)(p - s * Mc);
    const T* a = (const T*)args.a + block_offset(s, K, args.ncx, args.ncy, m);
    __syncthreads();
    for (int i = tid; i < m * m; i += blockDim.x) A[i] = ld(a, (i / m) * lda + (i % m));
    for (int i = tid; i < WN * WN; i += blockDim.x) Wn[i] = 0.0;
    for (int i = tid; i < WN * 3; i += blockDim.x) F[i] = 0.0;
    if (tid == 0) bad = 0;
    __syncthreads();
    if (osc && tid < 4) {
      // edge tid: its m edge-adjacent element values, the suffix sums of
      // their resistances, normalised
      const int ed = tid;
      auto ka = [&](int t) -> double {
        return ed == 0 ? A[t] : ed == 1 ? A[t * m + (m - 1)] : ed == 2 ? A[(m - 1) * m + t] : A[t * m];
      };
      double tot = 0.0;
      for (int t = 0; t < m; ++t) tot += 1.0 / ka(t);
      for (int t = 0; t <= m; ++t) {
        double r = 0.0;
        for (int u = t; u < m; ++u) r += 1.0 / ka(u);
        Gp[ed * (m + 1) + t] = r / tot;
      }
    }
    __syncthreads();
    // boundary value of data set l (< 3) at boundary node (qx, qy)
    auto gval = [&](int l, int qx, int qy) -> double {
      if (!osc) return pcorner(l, qx, qy, m);
      if (qy == 0) return l == 0 ? Gp[qx] : l == 1 ? 1.0 - Gp[qx] : 0.0;
      if (qx == m) return l == 1 ? Gp[(m + 1) + qy] : l == 2 ? 1.0 - Gp[(m + 1) + qy] : 0.0;
      if (qy == m) return l == 2 ? 1.0 - Gp[2 * (m + 1) + qx] : 0.0;  // corner 3 takes u, corner 2 takes 1 - u
      if (qx == 0) return l == 0 ? Gp[3 * (m + 1) + qy] : 0.0;         // corner 0 takes u, corner 3 takes 1 - u
      return 0.0;
    };

    // g . K_BB g' over the elements touching the boundary
    double sb[6] = {0, 0, 0, 0, 0, 0};
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int ex = e % m, ey = e / m;
      if (!(ex == 0 || ey == 0 || ex == m - 1 || ey == m - 1)) continue;
      if (!osc) {
        int q = 0;
        for (int l = 0; l < 3; ++l)
          for (int lp = l; lp < 3; ++lp) sb[q++] += A[e] * bb_coef(l, lp, ex, ey, m);
        continue;
      }
      // the element's boundary nodes (local order 0..3 counter-clockwise)
      double gv[3][4];
      bool onb[4];
      for (int al = 0; al < 4; ++al) {
        const int qx = ex + (al == 1 || al == 2), qy = ey + (al >= 2);
        onb[al] = qx == 0 || qx == m || qy == 0 || qy == m;
        for (int l = 0; l < 3; ++l) gv[l][al] = onb[al] ? gval(l, qx, qy) : 0.0;
      }
      int q = 0;
      for (int l = 0; l < 3; ++l)
        for (int lp = l; lp < 3; ++lp) {
          double t = 0.0;
          for (int al = 0; al < 4; ++al)
            for (int be = 0; be < 4; ++be)
              if (onb[al] && onb[be]) t += gv[l][al] * kref(al, be) * gv[lp][be];
          sb[q++] += A[e] * t;
        }
    }
    for (int q = 0; q < 6; ++q) {
      double v = sb[q];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((tid & 63) == 0) sbb_part[tid >> 6][q] = v;
    }

    // original row r of K_II and its right-hand sides; thread t < WN writes
    // the band entry at distance t from the diagonal, thread WN the rhs.
    auto insert_row = [&](int r) {
      const int ix = r % n, iy = r / n, px = ix + 1, py = iy + 1;
      const double aSW = A[iy * m + ix], aSE = A[iy * m + ix + 1];
      const double aNW = A[(iy + 1) * m + ix], aNE = A[(iy + 1) * m + ix + 1];
      if (tid <= B) {
        const int t = tid;
        double v = 0.0;
        if (t == 0) v += (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
        if (t == 1 && ix >= 1) v += -(aSW + aNW) * (1.0 / 6.0);
        if (t == n - 1 && iy >= 1 && ix <= n - 2) v += -aSE * (1.0 / 3.0);
        if (t == n && iy >= 1) v += -(aSW + aSE) * (1.0 / 6.0);
        if (t == n + 1 && iy >= 1 && ix >= 1) v += -aSW * (1.0 / 3.0);
        if (r - t >= 0) Wn[(r % WN) * WN + ((r - t) % WN)] = v;
      } else if (tid == B + 1) {
        double f[3] = {0, 0, 0};
        const int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
        const int dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
        const double ks[8] = {-(aSW + aNW) / 6.0, -(aSE + aNE) / 6.0, -(aSW + aSE) / 6.0, -(aNW + aNE) / 6.0,
                              -aSW / 3.0,         -aSE / 3.0,         -aNW / 3.0,         -aNE / 3.0};
        for (int q = 0; q < 8; ++q) {
          const int qx = px + dxs[q], qy = py + dys[q];
          if (qx == 0 || qx == m || qy == 0 || qy == m)
            for (int l = 0; l < 3; ++l) f[l] -= ks[q] * gval(l, qx, qy);
        }
        for (int l = 0; l < 3; ++l) F[(r % WN) * 3 + l] = f[l];
      }
    };

    for (int r = 0; r < (B < NI ? B : NI); ++r) insert_row(r);
    __syncthreads();
    double sc[6] = {0, 0, 0, 0, 0, 0};
    for (int j = 0; j < NI; ++j) {
      if (j + B < NI) {
        insert_row(j + B);
        __syncthreads();
      }
      const int jj = j % WN;
      const double d = Wn[jj * WN + jj];
      const double inv = 1.0 / d;
      const int cnt = (j + B < NI - 1 ? j + B : NI - 1) - j;
      const int npairs = cnt * (cnt + 1) / 2;
      for (int q = tid; q < npairs; q += blockDim.x) {
        int io = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
        while (io * (io + 1) / 2 > q) --io;
        while ((io + 1) * (io + 2) / 2 <= q) ++io;
        const int ko = q - io * (io + 1) / 2;
        const int i = j + 1 + io, k = j + 1 + ko;
        Wn[(i % WN) * WN + (k % WN)] -= Wn[(i % WN) * WN + jj] * inv * Wn[(k % WN) * WN + jj];
      }
      if (tid < cnt * 3) {
        const int i = j + 1 + tid / 3, l = tid % 3;
        F[(i % WN) * 3 + l] -= Wn[(i % WN) * WN + jj] * inv * F[jj * 3 + l];
      }
      if (tid == 0) {
        if (!(d > 0.0)) bad = 1;
        const double y0 = F[jj * 3], y1 = F[jj * 3 + 1], y2 = F[jj * 3 + 2];
        sc[0] += y0 * y0 * inv;
        sc[1] += y0 * y1 * inv;
        sc[2] += y0 * y2 * inv;
        sc[3] += y1 * y1 * inv;
        sc[4] += y1 * y2 * inv;
        sc[5] += y2 * y2 * inv;
      }
      __syncthreads();
    }
    if (tid == 0) {
      double t6[6];
      for (int q = 0; q < 6; ++q) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) v += sbb_part[w][q];
        t6[q] = v - sc[q];
      }
      const double s3[3][3] = {{t6[0], t6[1], t6[2]}, {t6[1], t6[3], t6[4]}, {t6[2], t6[4], t6[5]}};
      store_packed(args.S + p * 10, s3);
      if (args.status) args.status[p] = bad ? STOMSFEM_ENOTSPD : STOMSFEM_OK;
    }
  }
}

size_t upscale_ref_lds_bytes(int m) {
  const int WN = m + 1;
  return sizeof(double) * ((size_t)m * m + (size_t)WN * WN + (size_t)WN * 3 + 4 * (size_t)(m + 1));
}

hipError_t launch_upscale_ref(const UpArgs& args, int a_dtype, hipStream_t st) {
  const size_t lds = upscale_ref_lds_bytes(args.m);
  const int64_t blocks = args.npairs < 65536 ? args.npairs : 65536;
  if (blocks == 0) return hipSuccess;
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(upscale_ref_kernel<float>, dim3((unsigned)blocks), dim3(REF_THREADS), lds, st, args);
  else
    hipLaunchKernelGGL(upscale_ref_kernel<double>, dim3((unsigned)blocks), dim3(REF_THREADS), lds, st, args);
  return hipGetLastError();
}

}  // namespace stomsfem
