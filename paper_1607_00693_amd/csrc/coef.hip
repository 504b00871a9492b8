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

// One workgroup per 16 x 16 tile of one sample.  The oscillating factor is
// separable, sin(2 pi x/eps) sin(2 pi y/eps), so its sines are evaluated once
// per tile row and column (32 instead of 512 per tile) and shared in LDS;
// when the whole tile lies in one bump cell (always on meshes whose bump
// cells are a multiple of 16 elements wide) the candidate bumps are the same
// for every element, so the cell is passed as a uniform value; every value
// is computed by the same expressions as the per-element form.
constexpr int COEF_TILE = 16;

template <typename T>
__global__ __launch_bounds__(256) void coef_bumps_kernel(CoefArgs c, int tiles_x) {
  __shared__ double sx[COEF_TILE], sy[COEF_TILE];
  const int64_t tiles = (int64_t)tiles_x * tiles_x;
  const int64_t nblk = c.nsamples * tiles;
  const double h = 1.0 / c.nfine;
  const int lane = threadIdx.x;
  const BumpParams bp{c.g, c.rho, c.eps, c.base, c.amp, c.beta};
  // workgroup-uniform loop over (sample, tile): the grid is capped so that
  // the launch stays within the per-dispatch thread limit
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int64_t s = b / tiles;
    const int tt = (int)(b - s * tiles);
    const int tx = tt % tiles_x, ty = tt / tiles_x;
    __syncthreads();  // the previous tile's readers are done with sx, sy
    if (lane < COEF_TILE) {
      const double x = ((tx * COEF_TILE + lane) + 0.5) * h;
      sx[lane] = sin(2.0 * M_PI * x / c.eps);
    } else if (lane < 2 * COEF_TILE) {
      const double y = ((ty * COEF_TILE + lane - COEF_TILE) + 0.5) * h;
      sy[lane - COEF_TILE] = sin(2.0 * M_PI * y / c.eps);
    }
    __syncthreads();
    // the tile's first and last element centroids in each direction
    const int x1 = min(tx * COEF_TILE + COEF_TILE - 1, c.nfine - 1), y1 = min(ty * COEF_TILE + COEF_TILE - 1, c.nfine - 1);
    const int cx0 = bump_cell((tx * COEF_TILE + 0.5) * h, c.g), cx1 = bump_cell((x1 + 0.5) * h, c.g);
    const int cy0 = bump_cell((ty * COEF_TILE + 0.5) * h, c.g), cy1 = bump_cell((y1 + 0.5) * h, c.g);
    const bool one_cell = cx0 == cx1 && cy0 == cy1;
    const int ix = tx * COEF_TILE + (lane % COEF_TILE), iy = ty * COEF_TILE + lane / COEF_TILE;
    if (ix < c.nfine && iy < c.nfine) {
      const double x = (ix + 0.5) * h, y = (iy + 0.5) * h;
      const double field = one_cell ? bump_field_cell(x, y, c.xi + s * c.nxi, bp, cx0, cy0)
                                    : bump_field(x, y, c.xi + s * c.nxi, bp);
      const double osc = c.base + c.amp * sx[lane % COEF_TILE] * sy[lane / COEF_TILE];
      ((T*)c.a)[(s * c.nfine + iy) * (int64_t)c.nfine + ix] = (T)(osc * exp(c.beta * field));
    }
  }
}

hipError_t launch_coef_bumps(int64_t nsamples, int nfine, const double* xi, int nxi, int g, double rho, double eps,
                             double base, double amp, double beta, void* a, int a_dtype, hipStream_t st) {
  CoefArgs c{nsamples, nfine, nxi, g, rho, eps, base, amp, beta, xi, a};
  const int tiles_x = (nfine + COEF_TILE - 1) / COEF_TILE;
  int64_t blocks = nsamples * (int64_t)tiles_x * tiles_x;
  if (blocks == 0) return hipSuccess;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(coef_bumps_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, c, tiles_x);
  else
    hipLaunchKernelGGL(coef_bumps_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, c, tiles_x);
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
                                                            int64_t tiles, int64_t nblk, T* __restrict__ a) {
  __shared__ double th[FEAT_MAX];
  int64_t s_loaded = -1;
  // workgroup-uniform loop over (sample, tile) with a capped grid
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int64_t s = b / tiles;
    const int64_t e0 = (b - s * tiles) * FEAT_TILE;
    if (s != s_loaded) {
      __syncthreads();
      for (int j = threadIdx.x; j < nfeat; j += 256) th[j] = feature_theta(xi[s * nxi + j], decades);
      __syncthreads();
      s_loaded = s;
    }
    T* as = a + s * per;
    const int64_t e1 = min(e0 + FEAT_TILE, per);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      const int32_t f = map[e];
      as[e] = (T)((unsigned)f < (unsigned)nfeat ? th[f] : 1.0);
    }
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
  const int64_t nblk = nsamples * tiles;
  if (nblk == 0) return hipSuccess;
  const int64_t blocks = nblk < (1 << 20) ? nblk : (1 << 20);
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(coef_features_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, per, nfeat, map, xi,
                       nxi, decades, tiles, nblk, (float*)a);
  else
    hipLaunchKernelGGL(coef_features_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, per, nfeat, map, xi,
                       nxi, decades, tiles, nblk, (double*)a);
  return hipGetLastError();
}

}  // namespace stomsfem
