// Coefficient samples of the synthetic bump family: the exponential
// transform of Sec. 2.1.3 (eq. nonlinear1) applied to an affine sum of
// compactly supported local modes, times a periodic oscillation,
//   a(x, xi) = (base + amp sin(2 pi x1/eps) sin(2 pi x2/eps))
//              * exp(beta * sum_j xi_j psi_j(x)),
//   psi_j(x) = (1 - |x - c_j|^2/rho^2)^2 inside the disc of radius rho.
// One thread per fine element, sampled at the centroid.  Only bumps whose
// centre cell lies within ceil(rho*g) cells of the point are visited, in
// increasing j.
#include "common.h"

namespace stomsfem {

struct CoefArgs {
  int64_t nsamples;
  int32_t nfine, nxi, g;
  double rho, eps, base, amp, beta;
  const double* xi;
  void* a;
};

template <typename T>
__global__ __launch_bounds__(256) void coef_bumps_kernel(CoefArgs c) {
  const int64_t per = (int64_t)c.nfine * c.nfine;
  const int64_t total = c.nsamples * per;
  const double h = 1.0 / c.nfine;
  const BumpParams bp{c.g, c.rho, c.eps, c.base, c.amp, c.beta};
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = t / per;
    const int rem = (int)(t - s * per);
    const int iy = rem / c.nfine, ix = rem - iy * c.nfine;
    ((T*)c.a)[t] = (T)bump_coef((ix + 0.5) * h, (iy + 0.5) * h, c.xi + s * c.nxi, bp);
  }
}

hipError_t launch_coef_bumps(int64_t nsamples, int nfine, const double* xi, int nxi, int g, double rho, double eps,
                             double base, double amp, double beta, void* a, int a_dtype, hipStream_t st) {
  CoefArgs c{nsamples, nfine, nxi, g, rho, eps, base, amp, beta, xi, a};
  const int64_t total = nsamples * (int64_t)nfine * nfine;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 1 << 20) blocks = 1 << 20;
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(coef_bumps_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, c);
  else
    hipLaunchKernelGGL(coef_bumps_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, c);
  return hipGetLastError();
}

}  // namespace stomsfem

// ---------------------------------------------------------------------------
// High-contrast channels-and-inclusions medium.  The geometry does not
// depend on the sample, so it is rasterised once per resolution into a
// feature map (index of the highest feature covering each fine element, -1
// for the background); a sample's coefficient is then a gather of its
// feature conductivities theta_j = 10^(decades * sigmoid(xi_j)).
// Coverage (element centroid xc, yc; h = 1/nfine): kind 0 = horizontal
// channel on row floor(y0 nfine) with x0 <= xc <= x0 + size; kind 1 =
// vertical channel on column floor(x0 nfine) with y0 <= yc <= y0 + size;
// kind 2 = square of side `size` centred at (x0, y0), |xc-x0|, |yc-y0| <= size/2.
// ---------------------------------------------------------------------------
namespace stomsfem {

constexpr int FEAT_MAX = 1024;

__global__ __launch_bounds__(256) void feature_map_kernel(int32_t nfine, int32_t nfeat, const int32_t* __restrict__ kind,
                                                          const double* __restrict__ x0, const double* __restrict__ y0,
                                                          const double* __restrict__ size, int32_t* __restrict__ map) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)nfine * nfine) return;
  const int iy = (int)(t / nfine), ix = (int)(t - (int64_t)iy * nfine);
  const double h = 1.0 / nfine;
  const double xc = (ix + 0.5) * h, yc = (iy + 0.5) * h;
  int found = -1;
  for (int j = nfeat - 1; j >= 0 && found < 0; --j) {
    bool cover;
    if (kind[j] == 0) {
      const int row = min((int)floor(y0[j] * nfine), nfine - 1);
      cover = iy == row && xc >= x0[j] && xc <= x0[j] + size[j];
    } else if (kind[j] == 1) {
      const int col = min((int)floor(x0[j] * nfine), nfine - 1);
      cover = ix == col && yc >= y0[j] && yc <= y0[j] + size[j];
    } else {
      cover = fabs(xc - x0[j]) <= 0.5 * size[j] && fabs(yc - y0[j]) <= 0.5 * size[j];
    }
    if (cover) found = j;
  }
  map[t] = found;
}

constexpr int FEAT_TILE = 4096;  // fine elements per workgroup

template <typename T>
__global__ __launch_bounds__(256) void coef_features_kernel(int64_t per, int32_t nfeat, const int32_t* __restrict__ map,
                                                            const double* __restrict__ xi, int32_t nxi, double decades,
                                                            int64_t tiles, T* __restrict__ a) {
  __shared__ double th[FEAT_MAX];
  const int64_t s = blockIdx.x / tiles;
  const int64_t e0 = (blockIdx.x - s * tiles) * FEAT_TILE;
  for (int j = threadIdx.x; j < nfeat; j += 256) th[j] = pow(10.0, decades / (1.0 + exp(-xi[s * nxi + j])));
  __syncthreads();
  T* as = a + s * per;
  const int64_t e1 = min(e0 + FEAT_TILE, per);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int32_t f = map[e];
    as[e] = (T)((unsigned)f < (unsigned)nfeat ? th[f] : 1.0);
  }
}

hipError_t launch_feature_map(int nfine, int nfeat, const int32_t* kind, const double* x0, const double* y0,
                              const double* size, int32_t* map, hipStream_t st) {
  const int64_t n = (int64_t)nfine * nfine;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(feature_map_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nfine, nfeat, kind, x0,
                     y0, size, map);
  return hipGetLastError();
}

hipError_t launch_coef_features(int64_t nsamples, int nfine, const int32_t* map, int nfeat, const double* xi, int nxi,
                                double decades, void* a, int a_dtype, hipStream_t st) {
  const int64_t per = (int64_t)nfine * nfine;
  const int64_t tiles = (per + FEAT_TILE - 1) / FEAT_TILE;
  const int64_t blocks = nsamples * tiles;
  if (blocks == 0) return hipSuccess;
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(coef_features_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, per, nfeat, map, xi,
                       nxi, decades, tiles, (float*)a);
  else
    hipLaunchKernelGGL(coef_features_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, per, nfeat, map, xi,
                       nxi, decades, tiles, (double*)a);
  return hipGetLastError();
}

}  // namespace stomsfem
