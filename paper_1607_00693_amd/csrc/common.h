// Shared device-side definitions of the HIP path (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stomsfem.h"

namespace stomsfem {

// Arguments of one homogeneous upscaling batch, passed by value to kernels.
struct UpArgs {
  int64_t nsamples;
  int32_t ncx, ncy, m;
  int64_t npairs;     // nsamples * ncx * ncy
  const void* a;
  double* S;
  int32_t* status;
  int32_t bc;         // boundary data of the cell problems: 0 linear, 1 oscillatory (reference kernel only)
};

// Row-major offset of the m x m block of coarse element K of sample s.
__device__ __forceinline__ int64_t block_offset(int64_t s, int K, int ncx, int ncy, int m) {
  const int64_t lda = (int64_t)ncx * m;
  const int kx = K % ncx, ky = K / ncx;
  return s * ((int64_t)ncy * m) * lda + (int64_t)ky * m * lda + (int64_t)kx * m;
}

template <typename T>
__device__ __forceinline__ double ld(const T* p, int64_t i) {
  return (double)p[i];
}

// Bilinear corner functions p^l at the boundary node (px, py) of the m x m
// local grid, l = 0..2 (p^3 follows from the partition of unity).
__host__ __device__ constexpr double pcorner(int l, int px, int py, int m) {
  return l == 0   ? (1.0 - (double)px / m) * (1.0 - (double)py / m)
         : l == 1 ? ((double)px / m) * (1.0 - (double)py / m)
                  : ((double)px / m) * ((double)py / m);
}

// Q1 element matrix of int grad N_a . grad N_b on a square (unit coefficient),
// nodes counter-clockwise from the lower-left corner.
__host__ __device__ constexpr double kref(int a, int b) {
  return a == b ? 4.0 / 6.0 : ((a - b == 2 || b - a == 2) ? -2.0 / 6.0 : -1.0 / 6.0);
}

// Energy g_e^l . K_ref g_e^l' of one fine element whose nodes lying on the
// boundary of the coarse element carry the bilinear data p^l (interior nodes
// carry 0).  Element (ex, ey) of the m x m local grid.
__host__ __device__ constexpr double bb_coef(int l, int lp, int ex, int ey, int m) {
  double s = 0.0;
  for (int al = 0; al < 4; ++al) {
    const int pxa = ex + (al == 1 || al == 2), pya = ey + (al >= 2);
    const bool ba = pxa == 0 || pxa == m || pya == 0 || pya == m;
    if (!ba) continue;
    for (int be = 0; be < 4; ++be) {
      const int pxb = ex + (be == 1 || be == 2), pyb = ey + (be >= 2);
      const bool bb = pxb == 0 || pxb == m || pyb == 0 || pyb == m;
      if (!bb) continue;
      s += pcorner(l, pxa, pya, m) * kref(al, be) * pcorner(lp, pxb, pyb, m);
    }
  }
  return s;
}

// Write the packed 10 entries of S from its 3x3 block on l, l' < 3 using
// phi^3 = 1 - phi^0 - phi^1 - phi^2 (constants are a-harmonic, so S 1 = 0).
__device__ __forceinline__ void store_packed(double* out, const double s[3][3]) {
  const double s03 = -(s[0][0] + s[0][1] + s[0][2]);
  const double s13 = -(s[0][1] + s[1][1] + s[1][2]);
  const double s23 = -(s[0][2] + s[1][2] + s[2][2]);
  const double s33 = -(s03 + s13 + s23);
  out[0] = s[0][0];
  out[1] = s[0][1];
  out[2] = s[0][2];
  out[3] = s03;
  out[4] = s[1][1];
  out[5] = s[1][2];
  out[6] = s13;
  out[7] = s[2][2];
  out[8] = s23;
  out[9] = s33;
}

// Parameters of the synthetic bump coefficient family (see coef.hip).
struct BumpParams {
  int32_t g;
  double rho, eps, base, amp, beta;
};

// sum_j xi_j psi_j(x, y) of the bump family at the point (x, y), xs = this
// sample's xi.  Only bumps whose centre cell lies within ceil(rho*g) cells
// are visited, in increasing index order.
// (Multiplications by 1/g and 1/rho^2 replace the divisions: exact when g
// and rho are powers of two, within an ulp otherwise.)
// The same sum for a point whose centre cell (bx, by) the caller supplies
// (a workgroup whose points share one cell passes it as a uniform value, so
// the loop bounds and the xi loads are uniform too).
// XS: stride between consecutive xi_j in memory (1 for a sample's row of xi).
template <int XS = 1>
__device__ __forceinline__ double bump_field_cell(double x, double y, const double* xs, const BumpParams& bp, int bx,
                                                  int by) {
  const double ginv = 1.0 / bp.g, rinv2 = 1.0 / (bp.rho * bp.rho);
  const int reach = (int)ceil(bp.rho * bp.g);
  double field = 0.0;
  for (int jy = max(by - reach, 0); jy <= min(by + reach, bp.g - 1); ++jy) {
    const double cy = (jy + 0.5) * ginv, dy2 = (y - cy) * (y - cy);
    for (int jx = max(bx - reach, 0); jx <= min(bx + reach, bp.g - 1); ++jx) {
      const double cx = (jx + 0.5) * ginv;
      const double r2 = ((x - cx) * (x - cx) + dy2) * rinv2;
      if (r2 < 1.0) field += xs[(jy * bp.g + jx) * XS] * (1.0 - r2) * (1.0 - r2);
    }
  }
  return field;
}

// centre cell of a point along one axis
__device__ __forceinline__ int bump_cell(double x, int g) { return min((int)(x * g), g - 1); }

template <int XS = 1>
__device__ __forceinline__ double bump_field(double x, double y, const double* xs, const BumpParams& bp) {
  return bump_field_cell<XS>(x, y, xs, bp, bump_cell(x, bp.g), bump_cell(y, bp.g));
}

// Conductivity of feature j of the channels-and-inclusions medium:
// theta = 10^(decades sigmoid(xi_j)) (the bounded transform of Sec. 2.1.3).
// Every kernel that forms it uses this function, so they agree bit for bit.
__device__ __forceinline__ double feature_theta(double xi, double decades) {
  return pow(10.0, decades / (1.0 + exp(-xi)));
}

// a(x, xi) of the bump family at the point (x, y).
__device__ __forceinline__ double bump_coef(double x, double y, const double* xs, const BumpParams& bp) {
  const double field = bump_field(x, y, xs, bp);
  const double osc = bp.base + bp.amp * sin(2.0 * M_PI * x / bp.eps) * sin(2.0 * M_PI * y / bp.eps);
  return osc * exp(bp.beta * field);
}

}  // namespace stomsfem
