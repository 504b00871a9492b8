// Device helpers of the reduced basis on oversampled patches, shared by
// the FP64 online kernel (rb_os.hip) and the FP32 matrix-core online kernel
// (rb.hip).
#pragma once
#include "rb.h"

namespace stomsfem {

// first fine cell (one axis) of the patch of coarse element k: the patch of
// m + 2o cells centred on the element, moved inside [0, nf)
__host__ __device__ inline int rbo_origin(int k, int m, int o, int nf) {
  int x0 = k * m - o;
  if (x0 > nf - (m + 2 * o)) x0 = nf - (m + 2 * o);
  return x0 < 0 ? 0 : x0;
}

// c^l = -A^{-1} Fh_l (l = 0..2) from v = [A upper triangle | Fh] (any
// numeric type) by LDL^T in FP64, in place (d_j on the diagonal), with the
// identity on the unused modes q >= r.  False on a non-positive (or NaN)
// pivot.
template <int RMAX, typename TV>
__device__ __forceinline__ bool rbo_coeffs(const TV* v, int r, double c[3][RMAX]) {
  constexpr int NA = RMAX * (RMAX + 1) / 2;
  double L[RMAX][RMAX];
  bool ok = true;
#pragma unroll
  for (int q = 0; q < RMAX; ++q)
#pragma unroll
    for (int qp = q; qp < RMAX; ++qp) {
      const double a = (double)v[q * RMAX - q * (q - 1) / 2 + (qp - q)];
      L[qp][q] = (q < r && qp < r) ? a : (q == qp ? 1.0 : 0.0);
    }
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    double d = L[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k] * L[k][k];
    ok = ok && d > 0.0;
    L[j][j] = d;
    const double inv = 1.0 / d;
#pragma unroll
    for (int i = j + 1; i < RMAX; ++i) {
      double u = L[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) u -= L[i][k] * L[j][k] * L[k][k];
      L[i][j] = u * inv;
    }
  }
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    double x[RMAX];
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
      double s = (i < r) ? (double)v[NA + l * RMAX + i] : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) s -= L[i][k] * x[k];
      x[i] = s;
    }
#pragma unroll
    for (int i = RMAX - 1; i >= 0; --i) {
      double s = x[i] / L[i][i];
#pragma unroll
      for (int k = i + 1; k < RMAX; ++k) s -= L[k][i] * c[l][k];
      c[l][i] = s;
    }
#pragma unroll
    for (int i = 0; i < RMAX; ++i) c[l][i] = -c[l][i];
  }
  return ok;
}

// S16 = Psi^{-T} T from the coefficients c, the sums U[f][l'] (at Uf[4 f +
// l']) and the corner values Pc [4][NF] (Gaussian elimination with partial pivoting on Psi^T).
// False if Psi is singular.
template <int RMAX, typename TU>
__device__ __forceinline__ bool rbo_recombine(const double c[3][RMAX], const TU* Uf, const double* Pc,
                                              double S[4][4]) {
  double Tm[4][4], Pt[4][4];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int lp = 0; lp < 4; ++lp) {
      double s = (double)Uf[4 * j + lp];
#pragma unroll
      for (int q = 0; q < RMAX; ++q) s += c[j][q] * (double)Uf[4 * (3 + q) + lp];
      Tm[j][lp] = s;
    }
#pragma unroll
  for (int lp = 0; lp < 4; ++lp) Tm[3][lp] = -(Tm[0][lp] + Tm[1][lp] + Tm[2][lp]);
  // Pt = Psi^T: Pt[j][k] = psi^j(x_k)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double sum = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = Pc[k * RBO_NF + j];
#pragma unroll
      for (int q = 0; q < RMAX; ++q) s += c[j][q] * Pc[k * RBO_NF + 3 + q];
      Pt[j][k] = s;
      sum += s;
    }
    Pt[3][k] = 1.0 - sum;
  }
  // solve Pt S = Tm (every index compile-time: the row interchange is a
  // select per entry)
  bool sing = false;
#pragma unroll
  for (int col = 0; col < 4; ++col) {
    int pr = col;
    double best = fabs(Pt[col][col]);
#pragma unroll
    for (int i = col + 1; i < 4; ++i)
      if (fabs(Pt[i][col]) > best) {
        best = fabs(Pt[i][col]);
        pr = i;
      }
#pragma unroll
    for (int i = col + 1; i < 4; ++i) {
      const bool sw = i == pr;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const double a = Pt[col][cc], b = Tm[col][cc];
        Pt[col][cc] = sw ? Pt[i][cc] : a;
        Pt[i][cc] = sw ? a : Pt[i][cc];
        Tm[col][cc] = sw ? Tm[i][cc] : b;
        Tm[i][cc] = sw ? b : Tm[i][cc];
      }
    }
    sing = sing || !(fabs(Pt[col][col]) > 0.0);
    const double iv = 1.0 / Pt[col][col];
#pragma unroll
    for (int i = col + 1; i < 4; ++i) {
      const double f = Pt[i][col] * iv;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        Pt[i][cc] -= f * Pt[col][cc];
        Tm[i][cc] -= f * Tm[col][cc];
      }
    }
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    const double iv = 1.0 / Pt[i][i];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      double s = Tm[i][cc];
#pragma unroll
      for (int k = i + 1; k < 4; ++k) s -= Pt[i][k] * S[k][cc];
      S[i][cc] = s * iv;
    }
  }
  return !sing;
}

}  // namespace stomsfem
