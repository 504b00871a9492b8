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
