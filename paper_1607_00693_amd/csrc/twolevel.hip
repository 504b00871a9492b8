// Two-level Monte Carlo estimator (Sec. 4.1.1, the remark with eqs.
// MCmean2level and mseML): per interior coarse node i,
//   mean[i]  = (1/N_H) sum_s U_H[s][i] + (1/N_h) sum_s (u_h[s][f(i)] - U_Hh[s][i]),
//   var_H[i] = M[U_H^2] - M[U_H]^2,  var_d[i] = M[d^2] - M[d]^2,
// d = u_h - U_Hh, f(i) the fine interior node at coarse node (px, py):
// (py m - 1)(nc m - 1) + (px m - 1).  One workgroup per 64 nodes, sixteen
// wavefronts over the samples (each with four loads in flight), combined in
// order: a fixed summation order.
#include "common.h"

namespace stomsfem {

constexpr int TL_WAVES = 16;

__global__ __launch_bounds__(64 * TL_WAVES) void two_level_kernel(const double* __restrict__ UH, int64_t nH,
                                                        const double* __restrict__ UHh,
                                                        const double* __restrict__ uf, int64_t nh, int nc, int m,
                                                        double* __restrict__ mean, double* __restrict__ var_H,
                                                        double* __restrict__ var_d) {
  __shared__ double red[TL_WAVES][64][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n1 = nc - 1, nU = n1 * n1;
  const int i = blockIdx.x * 64 + lane;
  double s1H = 0.0, s2H = 0.0, s1d = 0.0, s2d = 0.0;
  if (i < nU) {
    const int px = i % n1 + 1, py = i / n1 + 1;
    const int64_t nf1 = (int64_t)nc * m - 1;
    const int64_t fi = (py * (int64_t)m - 1) * nf1 + (px * (int64_t)m - 1);
#pragma unroll 4
    for (int64_t s = wv; s < nH; s += TL_WAVES) {
      const double u = UH[s * nU + i];
      s1H += u;
      s2H += u * u;
    }
#pragma unroll 4
    for (int64_t s = wv; s < nh; s += TL_WAVES) {
      const double d = uf[s * nf1 * nf1 + fi] - UHh[s * nU + i];
      s1d += d;
      s2d += d * d;
    }
  }
  red[wv][lane][0] = s1H;
  red[wv][lane][1] = s2H;
  red[wv][lane][2] = s1d;
  red[wv][lane][3] = s2d;
  __syncthreads();
  if (wv == 0 && i < nU) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int v = 0; v < TL_WAVES; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) t[q] += red[v][lane][q];
    const double mH = t[0] / (double)nH, md = t[2] / (double)nh;
    if (mean) mean[i] = mH + md;
    if (var_H) var_H[i] = t[1] / (double)nH - mH * mH;
    if (var_d) var_d[i] = t[3] / (double)nh - md * md;
  }
}

hipError_t launch_two_level(const double* UH, int64_t nH, const double* UHh, const double* uf, int64_t nh, int nc,
                            int m, double* mean, double* var_H, double* var_d, hipStream_t st) {
  const int nU = (nc - 1) * (nc - 1);
  hipLaunchKernelGGL(two_level_kernel, dim3((unsigned)((nU + 63) / 64)), dim3(64 * TL_WAVES), 0, st, UH, nH, UHh, uf,
                     nh, nc, m,
                     mean, var_H, var_d);
  return hipGetLastError();
}

}  // namespace stomsfem
