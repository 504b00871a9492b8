// Per-lane local upscaling for m <= 8 (see upscale_small.hip for the
// mathematics); shared by the upscaling kernel and the surrogate fallback.
#pragma once
#include <type_traits>
#include <utility>

#include "common.h"

namespace stomsfem {

// Compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1, so
// that every index into the register window is a constant.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <int M, typename T>
struct SmallCell {
  static constexpr int n = M - 1;   // interior nodes per grid row
  static constexpr int NI = n * n;  // interior unknowns
  static constexpr int B = M;       // half-bandwidth (9-point stencil, natural order)
  static constexpr int WN = B + 1;  // window rows

  double W[WN][WN];    // entry (r, c), c <= r, stored at [r % WN][c % WN]
  double F[WN][3];     // right-hand sides, row r at [r % WN]
  double alo[M], ahi[M];  // element rows iy and iy+1 of the current fresh grid row
  double sbb[3][3];    // g . K_BB g'
  double sc[3][3];     // sum y y^T / d
  bool ok;

  const T* a;
  int64_t lda;

  __device__ __forceinline__ void load_elem_row(int ey, double* dst) {
    // keep the scheduler from hoisting every coefficient load of the fully
    // unrolled elimination to the top (that would hold all m*m values live)
    asm volatile("" ::: "memory");
#pragma unroll
    for (int ex = 0; ex < M; ++ex) dst[ex] = ld(a, ey * lda + ex);
    // boundary-boundary energy of the elements of this row that touch the boundary
#pragma unroll
    for (int ex = 0; ex < M; ++ex) {
      if (!(ey == 0 || ey == M - 1 || ex == 0 || ex == M - 1)) continue;
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int lp = l; lp < 3; ++lp) sbb[l][lp] += dst[ex] * bb_coef(l, lp, ex, ey, M);
    }
  }

  // Original matrix row r (node (ix, iy), grid node (ix+1, iy+1)) and its
  // right-hand sides -sum_{boundary neighbours} k_rb g^l_b.
  template <int r>
  __device__ __forceinline__ void insert_row() {
    constexpr int ix = r % n, iy = r / n;
    constexpr int px = ix + 1, py = iy + 1;
    if constexpr (ix == 0) {  // entering a new grid row: shift the element-row pair
      if constexpr (iy == 0) {
        load_elem_row(0, alo);
      } else {
#pragma unroll
        for (int e = 0; e < M; ++e) alo[e] = ahi[e];
      }
      load_elem_row(iy + 1, ahi);
    }
    const double aSW = alo[ix], aSE = alo[ix + 1], aNW = ahi[ix], aNE = ahi[ix + 1];
    const double diag = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
    const double cW = -(aSW + aNW) * (1.0 / 6.0), cE = -(aSE + aNE) * (1.0 / 6.0);
    const double cS = -(aSW + aSE) * (1.0 / 6.0), cN = -(aNW + aNE) * (1.0 / 6.0);
    const double cSW = -aSW * (1.0 / 3.0), cSE = -aSE * (1.0 / 3.0);
    const double cNW = -aNW * (1.0 / 3.0), cNE = -aNE * (1.0 / 3.0);
    constexpr int rr = r % WN;
#pragma unroll
    for (int c = (r - B > 0 ? r - B : 0); c <= r; ++c) W[rr][c % WN] = 0.0;
    W[rr][r % WN] = diag;
    double f[3] = {0.0, 0.0, 0.0};
    // neighbour (dx, dy) with coupling k: lower interior neighbours go into the
    // band, boundary neighbours into the right-hand sides, upper interior
    // neighbours are held by their own (later) rows.
    auto nb = [&](int dx, int dy, double k) __attribute__((always_inline)) {
      const int qx = px + dx, qy = py + dy;
      const bool bnd = qx == 0 || qx == M || qy == 0 || qy == M;
      if (bnd) {
#pragma unroll
        for (int l = 0; l < 3; ++l) f[l] -= k * pcorner(l, qx, qy, M);
      } else {
        const int c = (qy - 1) * n + (qx - 1);
        if (c < r) W[rr][c % WN] = k;
      }
    };
    nb(-1, 0, cW);
    nb(1, 0, cE);
    nb(0, -1, cS);
    nb(0, 1, cN);
    nb(-1, -1, cSW);
    nb(1, -1, cSE);
    nb(-1, 1, cNW);
    nb(1, 1, cNE);
#pragma unroll
    for (int l = 0; l < 3; ++l) F[rr][l] = f[l];
  }

  // Eliminate pivot j: rank-1 update of the window, forward substitution of
  // the right-hand sides, accumulation of y y^T / d.
  template <int j>
  __device__ __forceinline__ void eliminate() {
    constexpr int jj = j % WN;
    const double d = W[jj][jj];
    ok = ok && (d > 0.0);
    const double inv = 1.0 / d;
    constexpr int iend = (j + B < NI - 1) ? j + B : NI - 1;
    double t[WN], l[WN];
#pragma unroll
    for (int i = j + 1; i <= iend; ++i) {
      t[i - j] = W[i % WN][jj];
      l[i - j] = t[i - j] * inv;
    }
#pragma unroll
    for (int i = j + 1; i <= iend; ++i)
#pragma unroll
      for (int k = j + 1; k <= i; ++k) W[i % WN][k % WN] -= l[i - j] * t[k - j];
    const double y0 = F[jj][0], y1 = F[jj][1], y2 = F[jj][2];
#pragma unroll
    for (int i = j + 1; i <= iend; ++i) {
      F[i % WN][0] -= l[i - j] * y0;
      F[i % WN][1] -= l[i - j] * y1;
      F[i % WN][2] -= l[i - j] * y2;
    }
    const double z0 = y0 * inv, z1 = y1 * inv, z2 = y2 * inv;
    sc[0][0] += z0 * y0;
    sc[0][1] += z0 * y1;
    sc[0][2] += z0 * y2;
    sc[1][1] += z1 * y1;
    sc[1][2] += z1 * y2;
    sc[2][2] += z2 * y2;
  }

  __device__ __forceinline__ void run(double* out, int32_t* status) {
    ok = true;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int lp = 0; lp < 3; ++lp) sbb[l][lp] = sc[l][lp] = 0.0;
    if constexpr (NI == 0) {
      // m = 1: every node is a boundary node
      load_elem_row(0, alo);
    } else {
      static_for<0, (B < NI ? B : NI)>([&](auto r) { insert_row<decltype(r)::value>(); });
      static_for<0, NI>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (j + B < NI) insert_row<j + B>();
        eliminate<j>();
      });
    }
    double s[3][3];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int lp = l; lp < 3; ++lp) {
        s[l][lp] = sbb[l][lp] - sc[l][lp];
        s[lp][l] = s[l][lp];
      }
    store_packed(out, s);
    if (status) *status = ok ? STOMSFEM_OK : STOMSFEM_ENOTSPD;
  }
};

// Solve one pair: a points at its m x m coefficient block (row stride lda,
// global or LDS memory); out receives the 10 packed entries.
template <int M, typename T>
__device__ __forceinline__ void small_cell_solve(const T* a, int64_t lda, double* out, int32_t* status) {
  SmallCell<M, T> cell;
  cell.a = a;
  cell.lda = lda;
  cell.run(out, status);
}

}  // namespace stomsfem
