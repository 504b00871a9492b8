// Oversampled Petrov-Galerkin local upscaling, register-tiled (Sec. 2.2
// remark on oversampling; eq. stiffness_local_petrov) for patches of
// M = 4T fine cells per side, M = 16, 24, 32 (M = 16: oversampling ratio 2
// at H/h = 8; M = 32: ratio 2 at H/h = 16).
//
// Same quantities as upscale_os.hip (corner values psi^j(x_k) and Galerkin
// products A_jl = psi^j . K^K p^l as Schur products f^j . K_II^{-1} t with
// seven test vectors t carried beside the three lifts f^j), computed with the
// panel structure of upscale_tiled.hip: the live m x m window of the band is
// NT x NT tiles of T x T whose ten lower tiles sit in the registers of ten
// lanes (six pairs per wavefront, circular tile ownership, so no tile moves
// between lanes), and per panel of T pivots
//   1. T lanes build the entering rows (stencil, lifts, tests);
//   2. the lane holding the diagonal tile factors it, forward-substitutes
//      the ten columns of its rows and accumulates the 21 Schur products
//      f^jv . K_II^{-1} t (one column at a time: few registers), in its
//      registers for T = 4 and in the pair's LDS block for larger tiles;
//   3. the panel rows are solved against the unit factor by the ten lanes,
//      which also apply the panel to the rows' ten right-hand sides;
//   4. every lane applies the rank-T update to its tile.
// The right-hand sides of the live rows sit in a circular LDS ring.
#include "common.h"

namespace stomsfem {

#define OT_WAVE_SYNC()                                     \
  do {                                                     \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                       \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
  } while (0)

// The live window is NT x NT tiles; its NT(NT+1)/2 lower tiles sit in as
// many lanes of one pair (NT = 4: ten lanes, six pairs per wavefront; the
// 40- to 64-cell patches take T = 8 and NT = 5..8: 15 to 36 lanes, four to
// one pairs per wavefront; 60-cell patches T = 6 and NT = 10: 55 lanes).
template <int NT>
struct OtShape {
  static constexpr int G = NT * (NT + 1) / 2;  // lanes per pair
  static constexpr int SLOTS = 64 / G;         // pairs per wavefront
};
constexpr int OT_NV = 10;                // columns: lifts f^0..2, corner tests 0..3, r^0..2
constexpr int OT_NY = 21;                // Schur products f^jv . K_II^{-1} (column 3 + tv)
constexpr int OT_RED = 9 + 1;            // reduced over the lanes: boundary terms, bad flag

struct OtArgs {
  UpArgs up;
  int32_t o;
  // optional: solve only the pairs list[i], i < nlist, into S[i], status[i]
  const int64_t* list;
  int64_t nlist;
};

template <int T, int NT>
struct OtLdsCore {
  static constexpr int FW = NT * T;
  union {
    double pw[T][NT][T];                   // panel rows: pw[k][R'][i] = W(row R'*T+i of the panel, column k)
    double red[OtShape<NT>::G][OT_RED];    // final reduction (after the last panel)
  };
  double Y[OT_NY];            // Schur products f^jv . K_II^{-1} t, accumulated by the diagonal lane
  double L[T * (T - 1) / 2];  // strict lower part of the unit factor of the diagonal tile
  double invd[T];             // 1 / d_k
  double fr[T][2];            // entering rows: diagonal and W couplings
  double fx[4];               // entering rows: SE of rows T-2, T-1 and S of row T-1 (+ pad)
  double f[FW][OT_NV];        // right-hand sides of the live rows (circular); pivot rows hold D^{-1} y
};

template <int T, int NT>
struct OtLds : OtLdsCore<T, NT> {
  static constexpr int PADB = ((80 - (int)(sizeof(OtLdsCore<T, NT>) % 128)) + 128) % 128;
  char pad[PADB == 0 ? 128 : PADB];
};

__device__ __forceinline__ double ot_recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

// first fine cell (one axis) of the patch of coarse element k
__device__ __forceinline__ int ot_origin(int k, int m, int o, int nf) {
  int x0 = k * m - o;
  if (x0 > nf - (m + 2 * o)) x0 = nf - (m + 2 * o);
  return x0 < 0 ? 0 : x0;
}

// bilinear corner function p^l (l = 0..2) at (px, py), 1/size = rs
__device__ __forceinline__ double ot_pc(int l, int px, int py, double rs) {
  const double x = px * rs, y = py * rs;
  return l == 0 ? (1.0 - x) * (1.0 - y) : l == 1 ? x * (1.0 - y) : x * y;
}

// r^l = (K^K p^l) at patch node (px, py) from the coefficients of its four
// elements q4 = (SW, SE, NW, NE); only elements of K count (they see the node
// as local node 2, 3, 1, 0).
__device__ __forceinline__ double ot_rK(int l, int px, int py, int cx, int cy, int m, const double* q4) {
  const double rm = 1.0 / m;
  double v = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ex = px - 1 + (e & 1), ey = py - 1 + (e >> 1);
    if (ex < cx || ex >= cx + m || ey < cy || ey >= cy + m) continue;
    const int al = e == 0 ? 2 : e == 1 ? 3 : e == 2 ? 1 : 0;
    double s = 0.0;
#pragma unroll
    for (int be = 0; be < 4; ++be) {
      const int bx = ex + (be == 1 || be == 2), by = ey + (be >= 2);
      s += kref(al, be) * ot_pc(l, bx - cx, by - cy, rm);
    }
    v += q4[e] * s;
  }
  return v;
}

// T = 8 (M = 32 ... 64) runs one wavefront per SIMD: its tiles and ten
// right-hand sides take the whole register file (at M = 32, 256 VGPRs and
// about 100 AGPRs, no scratch; at two wavefronts per SIMD it spilled 444
// bytes per lane).
template <int M, int T, typename TA>
__global__ __launch_bounds__(64, (T >= 7 || M / T > 8) ? 1 : 2) void upscale_os_tiled_kernel(OtArgs args) {
  constexpr int NT = M / T, NV = OT_NV, OT_G = OtShape<NT>::G, OT_SLOTS = OtShape<NT>::SLOTS;
  static_assert(M == NT * T, "window must be NT x NT tiles");
  constexpr int n = M - 1, NI = n * n, NP = (NI + T - 1) / T;
  constexpr int FW = NT * T;
  using Lds = OtLds<T, NT>;
  __shared__ Lds lds_all[OT_SLOTS];

  const int lane = threadIdx.x & 63;
  if (lane >= OT_SLOTS * OT_G) return;
  const int q = lane / OT_G, g = lane - q * OT_G;
  Lds& sh = lds_all[q];
  // lane g of the pair owns the residue pair {P, Q}, Q <= P < NT, g = P(P+1)/2 + Q
  int P = 0;
  while ((P + 1) * (P + 2) / 2 <= g) ++P;
  const int Q = g - P * (P + 1) / 2;

  const int64_t nout = args.list ? args.nlist : args.up.npairs;
  int64_t io = (int64_t)blockIdx.x * OT_SLOTS + q;  // output slot
  const bool valid = io < nout;
  if (!valid) io = nout - 1;
  const int64_t p = args.list ? args.list[io] : io;
  const int m = args.up.m, o = args.o;
  const int ncx = args.up.ncx, ncy = args.up.ncy, Mc = ncx * ncy;
  const int64_t s = p / Mc;
  const int K = (int)(p - s * Mc), kx = K % ncx, ky = K / ncx;
  const int nfx = ncx * m, nfy = ncy * m;
  const int x0 = ot_origin(kx, m, o, nfx), y0 = ot_origin(ky, m, o, nfy);
  const int cx = kx * m - x0, cy = ky * m - y0;  // K's lower-left node in patch nodes
  const TA* a = (const TA*)args.up.a + s * (int64_t)nfy * nfx + (int64_t)y0 * nfx + x0;
  constexpr double rM = 1.0 / M;

  double tile[T][T];
  // small tiles leave room for the Schur products in registers (the diagonal
  // lane's critical path then has no LDS round trip for them); larger tiles
  // accumulate them in LDS, one writer per panel
  constexpr bool YR = T <= 4;
  double Yr[YR ? OT_NY : 1];
#pragma unroll
  for (int t = 0; t < (YR ? OT_NY : 1); ++t) Yr[t] = 0.0;
  for (int t = g; t < OT_NY; t += OT_G) sh.Y[t] = 0.0;
  bool bad = false;

  // coefficients of the four elements around the node of row r (patch frame)
  auto load_quad = [&](int r, double* q4) {
    if (r < NI) {
      const int ix = r % n, iy = r / n;
      q4[0] = ld(a, (int64_t)iy * nfx + ix);
      q4[1] = ld(a, (int64_t)iy * nfx + ix + 1);
      q4[2] = ld(a, (int64_t)(iy + 1) * nfx + ix);
      q4[3] = ld(a, (int64_t)(iy + 1) * nfx + ix + 1);
    } else {
      q4[0] = q4[1] = q4[2] = q4[3] = 0.0;
    }
  };
  // stencil row r (tile row i) into sh.fr / sh.fx, its ten right-hand sides
  // into sh.f (or rhs_out for rows entering during a panel); fr[] returns
  // (D, W, SE, S, SW) to the caller.  Rows past NI are identity rows.
  auto build_row = [&](int r, int i, const double* q4, double* fr, double* rhs_out) {
    fr[0] = 1.0;
    fr[1] = fr[2] = fr[3] = fr[4] = 0.0;
    double rhs[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) rhs[v] = 0.0;
    if (r < NI) {
      const int ix = r % n, iy = r / n, px = ix + 1, py = iy + 1;
      const double aSW = q4[0], aSE = q4[1], aNW = q4[2], aNE = q4[3];
      fr[0] = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
      constexpr int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
      constexpr int dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
      const double ks[8] = {-(aSW + aNW) * (1.0 / 6.0), -(aSE + aNE) * (1.0 / 6.0), -(aSW + aSE) * (1.0 / 6.0),
                            -(aNW + aNE) * (1.0 / 6.0), -aSW * (1.0 / 3.0),         -aSE * (1.0 / 3.0),
                            -aNW * (1.0 / 3.0),         -aNE * (1.0 / 3.0)};
      // lifts f^v = -sum over the patch-boundary neighbours of K[r][q] g^v(q)
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int qx = px + dxs[d], qy = py + dys[d];
        const bool bnd = qx == 0 || qx == M || qy == 0 || qy == M;
        const double k = bnd ? ks[d] : 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) rhs[l] -= k * ot_pc(l, qx, qy, rM);
      }
      // corner tests: the unit vector of each corner of K inside the patch
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int kpx = cx + ((k == 1 || k == 2) ? m : 0), kpy = cy + (k >= 2 ? m : 0);
        rhs[3 + k] = (px == kpx && py == kpy) ? 1.0 : 0.0;
      }
      if (px >= cx && px <= cx + m && py >= cy && py <= cy + m) {
#pragma unroll
        for (int l = 0; l < 3; ++l) rhs[7 + l] = ot_rK(l, px, py, cx, cy, m, q4);
      }
      fr[1] = ix >= 1 ? ks[0] : 0.0;
      fr[2] = (iy >= 1 && ix <= n - 2) ? ks[5] : 0.0;
      fr[3] = iy >= 1 ? ks[2] : 0.0;
      fr[4] = (iy >= 1 && ix >= 1) ? ks[4] : 0.0;
    }
    sh.fr[i][0] = fr[0];
    sh.fr[i][1] = fr[1];
    if (i == T - 2) sh.fx[0] = fr[2];
    if (i == T - 1) {
      sh.fx[1] = fr[2];
      sh.fx[2] = fr[3];
    }
    if (rhs_out) {
#pragma unroll
      for (int v = 0; v < NV; ++v) rhs_out[v] = rhs[v];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) sh.f[r % FW][v] = rhs[v];
    }
  };
  // original values of tile (row tile rt, column tile rt - dt) from sh.fr
  auto fresh_tile = [&](int dt) {
    const bool d0 = dt == 0, d1 = dt == 1, dl = dt == NT - 1;
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
      for (int k = 0; k < T; ++k) tile[i][k] = 0.0;
#pragma unroll
    for (int i = 0; i < T; ++i) {
      tile[i][i] = d0 ? sh.fr[i][0] : 0.0;
      if (i >= 1) tile[i][i - 1] = d0 ? sh.fr[i][1] : 0.0;
    }
    tile[0][T - 1] = d1 ? sh.fr[0][1] : 0.0;
    static_assert(T >= 3 && NT >= 3 && T * (NT - 1) == M - T, "band edge inside one tile column");
    tile[T - 2][0] = dl ? sh.fx[0] : 0.0;
    tile[T - 1][1] = dl ? sh.fx[1] : 0.0;
    tile[T - 1][0] = dl ? sh.fx[2] : 0.0;
  };

  // ---- initial window ----
  {
    const int R0 = P, C0 = Q;
    double q4[4];
    for (int rt = 0; rt < NT; ++rt) {
      if (g < T) {
        double frv[5];
        load_quad(T * rt + g, q4);
        build_row(T * rt + g, g, q4, frv, nullptr);
      }
      OT_WAVE_SYNC();
      if (R0 == rt) fresh_tile(R0 - C0);
      OT_WAVE_SYNC();
    }
  }

  double q4n[4];
  if (g < T) load_quad(T * NT + g, q4n);

  double ent[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) ent[v] = 0.0;
  for (int J = 0; J < NP; ++J) {
    const int j0 = J % NT;
    const int wP = J + ((P - j0 + NT) % NT), wQ = J + ((Q - j0 + NT) % NT);
    const int R = wP > wQ ? wP : wQ, C = wP > wQ ? wQ : wP;

    // 1. rows entering with row tile J + NT
    if (g < T) {
      const int r = T * (J + NT) + g;
      double q4[4] = {q4n[0], q4n[1], q4n[2], q4n[3]};
      if (J + 1 < NP) load_quad(r + T, q4n);
      double frv[5];
      build_row(r, g, q4, frv, ent);
#pragma unroll
      for (int k = 0; k < T; ++k) {
        double v = 0.0;
        if (k == g) v = frv[4];
        else if (k == g + 1) v = frv[3];
        else if (k == g + 2) v = frv[2];
        sh.pw[k][NT - 1][g] = v;
      }
    }
    // 2. diagonal tile: LDL^T in registers, then the ten columns of its rows
    //    one at a time: y = L^{-1} f, D^{-1} y to the ring, Schur products
    if (R == J && C == J) {
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const double d = tile[k][k];
        bad = bad || !(d > 0.0);
        const double inv = ot_recip(d);
        sh.invd[k] = inv;
#pragma unroll
        for (int i = k + 1; i < T; ++i) {
          const double li = tile[i][k] * inv;
#pragma unroll
          for (int c = k + 1; c <= i; ++c) tile[i][c] -= li * tile[c][k];
        }
#pragma unroll
        for (int i = k + 1; i < T; ++i) {
          tile[i][k] *= inv;
          sh.L[i * (i - 1) / 2 + k] = tile[i][k];
        }
      }
      double zf[T][3];  // D^{-1} y of the lifts
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double col[T];
#pragma unroll
        for (int k = 0; k < T; ++k) {
          double x = sh.f[(T * J + k) % FW][v];
#pragma unroll
          for (int kk = 0; kk < k; ++kk) x -= tile[k][kk] * col[kk];
          col[k] = x;
        }
        double y3[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < T; ++k) {
          const double z = col[k] * sh.invd[k];
          if (v < 3) {
            zf[k][v] = z;
          } else {
#pragma unroll
            for (int jv = 0; jv < 3; ++jv) y3[jv] += zf[k][jv] * col[k];
          }
          sh.f[(T * J + k) % FW][v] = z;
        }
        if (v >= 3) {
#pragma unroll
          for (int jv = 0; jv < 3; ++jv) {
            if constexpr (YR)
              Yr[jv * 7 + (v - 3)] += y3[jv];
            else
              sh.Y[jv * 7 + (v - 3)] += y3[jv];
          }
        }
      }
    } else if (C == J) {
      // 3a. sub-diagonal panel tile (R, J) -> panel rows (R-J-1)*T ...
      const int rb = R - J - 1;
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int k = 0; k < T; ++k) sh.pw[k][rb][i] = tile[i][k];
    }
    OT_WAVE_SYNC();
    // 3b. panel rows: W = A L^{-T}; rhs -= W (D^{-1} y) for the ten columns.
    //     Lane g < T solves the entering row NE + g last, from and into its
    //     registers; the other NE rows go round the lanes.
    {
      constexpr int NR = NT * T, NE = NR - T, RPL = (NR + OT_G - 1) / OT_G;
      static_assert(T * (RPL - 1) + (OT_G - T) * RPL >= NE, "panel rows fit the lanes");
#pragma unroll 1
      for (int t = 0; t < RPL; ++t) {
        const bool last = t == RPL - 1;
        const bool entering = last && g < T;
        const int rho0 = !last ? OT_G * t + g : (g < T ? NE + g : OT_G * t + g - T);
        const bool ok = entering || rho0 < NE;
        const int rho = ok ? rho0 : 0;
        double w[T];
#pragma unroll
        for (int k = 0; k < T; ++k) w[k] = sh.pw[k][rho / T][rho % T];
#pragma unroll
        for (int k = 1; k < T; ++k)
#pragma unroll
          for (int kk = 0; kk < k; ++kk) w[k] -= w[kk] * sh.L[k * (k - 1) / 2 + kk];
        double* fr = sh.f[(T * (J + 1) + rho) % FW];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double fa = entering ? ent[v] : fr[v];
#pragma unroll
          for (int k = 0; k < T; ++k) fa -= w[k] * sh.f[(T * J + k) % FW][v];
          if (ok) {
            if (entering) ent[v] = fa;
            else fr[v] = fa;
          }
        }
        if (ok) {
#pragma unroll
          for (int k = 0; k < T; ++k) sh.pw[k][rho / T][rho % T] = w[k];
        }
      }
    }
    // 4a. lanes whose tile left through the panel take the entering tile
    int Rn = R, Cn = C;
    if (C == J) {
      Rn = J + NT;
      Cn = (R == J) ? J + NT : R;
      fresh_tile(Rn - Cn);
    }
    OT_WAVE_SYNC();
    // the entering rows' right-hand sides take the retired pivot slots
    if (g < T) {
      double* fe = sh.f[(T * (J + NT) + g) % FW];
#pragma unroll
      for (int v = 0; v < NV; ++v) fe[v] = ent[v];
    }
    // 4b. trailing update of the new window [J+1, J+NT]
    {
      const int rb = Rn - J - 1, cb = Cn - J - 1;
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const double inv = sh.invd[k];
        double wr[T], zc[T];
#pragma unroll
        for (int i = 0; i < T; ++i) wr[i] = sh.pw[k][rb][i];
#pragma unroll
        for (int c = 0; c < T; ++c) zc[c] = sh.pw[k][cb][c] * inv;
#pragma unroll
        for (int i = 0; i < T; ++i)
#pragma unroll
          for (int c = 0; c < T; ++c) tile[i][c] -= wr[i] * zc[c];
      }
    }
    OT_WAVE_SYNC();
  }

  // ---- g^j . r^l over K's nodes on the patch boundary (K touches it only at
  //      the edges of the domain, where the patch is moved inside) ----
  double bt[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) bt[t] = 0.0;
  for (int id = g; id < (m + 1) * (m + 1); id += OT_G) {
    const int ax = cx + id % (m + 1), ay = cy + id / (m + 1);
    if (!(ax == 0 || ax == M || ay == 0 || ay == M)) continue;
    double q4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ex = ax - 1 + (e & 1), ey = ay - 1 + (e >> 1);
      const bool inside = ex >= 0 && ex < M && ey >= 0 && ey < M;
      q4[e] = inside ? ld(a, (int64_t)(inside ? ey : 0) * nfx + (inside ? ex : 0)) : 0.0;
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double rl = ot_rK(l, ax, ay, cx, cy, m, q4);
#pragma unroll
      for (int jb = 0; jb < 3; ++jb) bt[3 * jb + l] += ot_pc(jb, ax, ay, rM) * rl;
    }
  }

  // ---- reduce the ten lanes' boundary terms and flags through LDS, then
  //      lane 0 of the pair forms the 4x4 recombination ----
  if constexpr (YR) {
    // the diagonal lanes (P == Q) add their register sums in turn
#pragma unroll 1
    for (int h = 0; h < NT; ++h) {
      if (P == Q && P == h) {
#pragma unroll
        for (int t = 0; t < OT_NY; ++t) sh.Y[t] += Yr[t];
      }
      OT_WAVE_SYNC();
    }
  }
  double tot[OT_RED];
#pragma unroll
  for (int t = 0; t < 9; ++t) sh.red[g][t] = bt[t];
  sh.red[g][OT_RED - 1] = bad ? 1.0 : 0.0;
  OT_WAVE_SYNC();
  if (g == 0) {
#pragma unroll
    for (int t = 0; t < OT_RED; ++t) {
      double v = 0.0;
      for (int h = 0; h < OT_G; ++h) v += sh.red[h][t];
      tot[t] = v;
    }
  }
  if (g == 0 && valid) {
    double Ys[OT_NY];
#pragma unroll
    for (int t = 0; t < OT_NY; ++t) Ys[t] = sh.Y[t];
    const double* Bs = tot;
    const bool anybad = tot[OT_RED - 1] != 0.0;
    double Psi[4][4], A[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int kpx = cx + ((k == 1 || k == 2) ? m : 0), kpy = cy + (k >= 2 ? m : 0);
      const bool onb = kpx == 0 || kpx == M || kpy == 0 || kpy == M;
      double sum = 0.0;
#pragma unroll
      for (int jb = 0; jb < 3; ++jb) {
        Psi[k][jb] = onb ? ot_pc(jb, kpx, kpy, rM) : Ys[jb * 7 + k];
        sum += Psi[k][jb];
      }
      Psi[k][3] = 1.0 - sum;
    }
#pragma unroll
    for (int jb = 0; jb < 3; ++jb) {
      double rs = 0.0;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        A[jb][l] = Bs[3 * jb + l] + Ys[jb * 7 + 4 + l];
        rs += A[jb][l];
      }
      A[jb][3] = -rs;
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) A[3][l] = -(A[0][l] + A[1][l] + A[2][l]);
    // C = (Psi^T)^{-1}: Gauss-Jordan with partial pivoting on [Psi^T | I]
    // (every index compile-time: the row interchange is a select per entry)
    double G[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) G[i][c] = c < 4 ? Psi[c][i] : (c - 4 == i ? 1.0 : 0.0);
    bool sing = false;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int pr = c;
      double best = fabs(G[c][c]);
#pragma unroll
      for (int i = c + 1; i < 4; ++i)
        if (fabs(G[i][c]) > best) {
          best = fabs(G[i][c]);
          pr = i;
        }
#pragma unroll
      for (int i = c + 1; i < 4; ++i) {
        const bool sw = i == pr;
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          const double t = G[c][cc];
          G[c][cc] = sw ? G[i][cc] : t;
          G[i][cc] = sw ? t : G[i][cc];
        }
      }
      sing = sing || !(fabs(G[c][c]) > 0.0);
      const double iv = 1.0 / G[c][c];
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) G[c][cc] *= iv;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i == c) continue;
        const double f = G[i][c];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) G[i][cc] -= f * G[c][cc];
      }
    }
    double* out = args.up.S + io * 16;
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
      for (int lp = 0; lp < 4; ++lp) {
        double v = 0.0;
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) v += G[l][4 + jb] * A[jb][lp];
        out[4 * l + lp] = v;
      }
    if (args.up.status) args.up.status[io] = (anybad || sing) ? STOMSFEM_ENOTSPD : STOMSFEM_OK;
  }
}

// patches of 16, 20, 24 and 28 cells (T = 4 ... 7, NT = 4), of 32 to 64
// cells in steps of 8 (T = 8, NT = 4 ... 8), of 30, 36, 42, 54 and 60 cells
// (T = 6, NT = 5, 6, 7, 9, 10: up to 55 lanes per pair; ratio 3 at H/h = 10
// ... 20), of 25, 35, 45 and 50 cells (T = 5, NT = 5, 7, 9, 10) and of 49
// and 63 cells (T = 7, NT = 7, 9)
bool upscale_os_tiled_supports(int m, int o) {
  const int M = m + 2 * o;
  if (M >= 32 && M <= 64 && M % 8 == 0) return true;
  switch (M) {
    case 16: case 20: case 24: case 25: case 28: case 30: case 35: case 36: case 42: case 45: case 49: case 50:
    case 54: case 60: case 63: return true;
    default: return false;
  }
}

template <int M, int T>
static void launch_ot(const OtArgs& args, int a_dtype, hipStream_t st) {
  constexpr int SLOTS = OtShape<M / T>::SLOTS;
  const int64_t blocks = ((args.list ? args.nlist : args.up.npairs) + SLOTS - 1) / SLOTS;
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL((upscale_os_tiled_kernel<M, T, float>), dim3((unsigned)blocks), dim3(64), 0, st, args);
  else
    hipLaunchKernelGGL((upscale_os_tiled_kernel<M, T, double>), dim3((unsigned)blocks), dim3(64), 0, st, args);
}

hipError_t launch_upscale_os_tiled(const UpArgs& up, int o, int a_dtype, hipStream_t st, const int64_t* list,
                                   int64_t nlist) {
  if (!upscale_os_tiled_supports(up.m, o)) return hipErrorInvalidValue;
  if ((list ? nlist : up.npairs) <= 0) return hipSuccess;
  const OtArgs args{up, o, list, nlist};
  switch (up.m + 2 * o) {
    case 16: launch_ot<16, 4>(args, a_dtype, st); break;
    case 20: launch_ot<20, 5>(args, a_dtype, st); break;
    case 24: launch_ot<24, 6>(args, a_dtype, st); break;
    case 25: launch_ot<25, 5>(args, a_dtype, st); break;
    case 28: launch_ot<28, 7>(args, a_dtype, st); break;
    case 30: launch_ot<30, 6>(args, a_dtype, st); break;
    case 32: launch_ot<32, 8>(args, a_dtype, st); break;
    case 35: launch_ot<35, 5>(args, a_dtype, st); break;
    case 36: launch_ot<36, 6>(args, a_dtype, st); break;
    case 40: launch_ot<40, 8>(args, a_dtype, st); break;
    case 42: launch_ot<42, 6>(args, a_dtype, st); break;
    case 45: launch_ot<45, 5>(args, a_dtype, st); break;
    case 48: launch_ot<48, 8>(args, a_dtype, st); break;
    case 49: launch_ot<49, 7>(args, a_dtype, st); break;
    case 50: launch_ot<50, 5>(args, a_dtype, st); break;
    case 54: launch_ot<54, 6>(args, a_dtype, st); break;
    case 56: launch_ot<56, 8>(args, a_dtype, st); break;
    case 60: launch_ot<60, 6>(args, a_dtype, st); break;
    case 63: launch_ot<63, 7>(args, a_dtype, st); break;
    default: launch_ot<64, 8>(args, a_dtype, st); break;
  }
  return hipGetLastError();
}

}  // namespace stomsfem
