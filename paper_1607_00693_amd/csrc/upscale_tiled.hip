// Local upscaling for m = 16 and m = 32: register-tiled sliding-window LDL^T.
//
// Mathematics as in upscale_small.hip (Sec. 2.2 eqs. MsFEB and
// stiffness_local): S_ll' = g^l.K_BB g^l' - sum_j y_j^l y_j^l' / d_j with
// K_II = L D L^T and y = L^{-1} f, f^l = -K_IB g^l, so the factor is consumed
// as it is produced and never stored.
//
// Layout.  The band of K_II (natural order, half-bandwidth m) is eliminated
// in panels of T columns.  The live part of the band after a panel is an
// m x m window = NT x NT tiles of T x T (NT = 4).  Its NT(NT+1)/2 = 10
// lower-triangle tiles are held in the registers of 10 lanes; a wavefront
// serves 6 (element, sample) pairs.  Tile ownership is circular: the lane
// for the residue pair {P, Q} (mod NT) holds whichever of the tiles with row
// and column indices congruent to P and Q lies in the lower triangle of the
// current window.  When the window slides by one tile the only tiles that
// change owner are those leaving through the panel, and their lanes take
// over the tiles entering at the bottom, so no tile ever moves between
// lanes.  Per panel:
//   1. T lanes build the entering matrix rows (9-point stencil from the
//      coefficient block, Dirichlet lifts as right-hand sides);
//   2. the lane holding the diagonal tile factors it in registers (LDL^T),
//      forward-substitutes the right-hand sides and accumulates y y^T / d;
//   3. the lanes holding the sub-diagonal panel tiles publish them in LDS;
//      each of the 10 lanes solves a few panel rows against the unit L;
//   4. every lane applies the rank-T update W_R D^{-1} W_C^T to its tile.
// Communication inside a wavefront only (LDS plus wave-level ordering).
#include "common.h"
#include "small_cell.h"

namespace stomsfem {

#define WAVE_SYNC()                                    \
  do {                                                 \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                   \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
  } while (0)

constexpr int TL_NT = 4;               // tiles per window side
constexpr int TL_G = 10;               // lanes per pair = NT (NT + 1) / 2
constexpr int TL_SLOTS = 64 / TL_G;    // pairs per wavefront (6)

// Per-pair LDS block, kept small: occupancy is limited by LDS (eight
// wavefronts per CU at m = 32, 19.7 KB each).  TL_PAD > 0 would stagger the panel row
// blocks over the LDS banks, but costs one wavefront per CU, which was
// measured to matter more.  The block size is padded to 80 mod 128 bytes so
// that the six pairs of a wavefront start on different banks.
constexpr int TL_PAD = 0;

template <int M, int T>
struct TiledLdsCore {
  static constexpr int NT = TL_NT;
  static constexpr int FW = NT * T;  // rhs window rows
  union {
    double pw[T][NT][T + TL_PAD];  // panel rows: pw[k][R'][i] = W(row R'*T+i of the panel, column k)
    double red[TL_G][13];          // final reduction (after the last panel)
  };
  double L[T * (T - 1) / 2];  // strict lower part of the unit factor of the diagonal tile, row-packed
  double invd[T];             // 1 / d_k
  double fr[T][2];            // entering rows: diagonal and W couplings
  double fx[4];               // entering rows: SE of rows T-2, T-1 and S of row T-1 (+ pad)
  double f[FW][3];            // right-hand sides of the live rows (circular); the pivot
                              // rows' slots hold D^{-1} y once the diagonal tile is factored.
                              // Rows entering during a panel keep theirs in registers until
                              // the panel is solved, then take the retired pivot rows' slots.
};

template <int M, int T>
struct TiledLds : TiledLdsCore<M, T> {
  static constexpr int PADB = ((80 - (int)(sizeof(TiledLdsCore<M, T>) % 128)) + 128) % 128;
  char pad[PADB == 0 ? 128 : PADB];
};

// 1/d by Newton's iteration on the hardware reciprocal estimate (two steps
// take the estimate to full double precision).
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

// One wavefront's tile of TL_SLOTS pairs: pairs wtile * TL_SLOTS + q, q <
// TL_SLOTS; lds = the wavefront's TL_SLOTS per-pair blocks.  Lanes past the
// ten-lane groups return at once.
template <int M, int T, typename TA>
__device__ __forceinline__ void tiled_wave(const UpArgs& args, int64_t wtile, int lane, TiledLds<M, T>* lds) {
  constexpr int NT = TL_NT;
  static_assert(M == NT * T, "window must be NT x NT tiles");
  constexpr int n = M - 1, NI = n * n, NP = (NI + T - 1) / T;
  constexpr int FW = NT * T;
  using Lds = TiledLds<M, T>;

  if (lane >= TL_SLOTS * TL_G) return;
  const int q = lane / TL_G, g = lane - q * TL_G;
  Lds& sh = lds[q];
  // residue pair {P, Q}, P >= Q, of this lane: g = P (P + 1) / 2 + Q
  const int P = g >= 6 ? 3 : g >= 3 ? 2 : g >= 1 ? 1 : 0;
  const int Q = g - P * (P + 1) / 2;

  int64_t p = wtile * TL_SLOTS + q;
  const bool valid = p < args.npairs;
  if (!valid) p = args.npairs - 1;
  const int Mc = args.ncx * args.ncy;
  const int64_t s = p / Mc;
  const int K = (int)(p - s * Mc);
  const TA* a = (const TA*)args.a + block_offset(s, K, args.ncx, args.ncy, M);
  const int64_t lda = (int64_t)args.ncx * M;

  double tile[T][T];
  double sc[6] = {0, 0, 0, 0, 0, 0};
  bool bad = false;

  // ---- entering rows: lane g < T builds row r = T*rt + g ----
  // coefficient values of the four elements around the node of row r
  auto load_quad = [&](int r, double* q4) {
    if (r < NI) {
      const int ix = r % n, iy = r / n;
      q4[0] = ld(a, iy * lda + ix);
      q4[1] = ld(a, iy * lda + ix + 1);
      q4[2] = ld(a, (iy + 1) * lda + ix);
      q4[3] = ld(a, (iy + 1) * lda + ix + 1);
    } else {
      q4[0] = q4[1] = q4[2] = q4[3] = 0.0;
    }
  };
  // stencil row r (tile row i): diagonal and W coupling into sh.fr[i], the
  // far-band couplings SE, S of the last two rows into sh.fx, right-hand
  // sides into sh.f (or into rhs_out for rows entering during a panel);
  // fr[] returns (D, W, SE, S, SW) to the caller.
  auto build_row = [&](int r, int i, const double* q4, double* fr, double* rhs_out) {
    fr[0] = 1.0;
    fr[1] = fr[2] = fr[3] = fr[4] = 0.0;
    double rhs[3] = {0.0, 0.0, 0.0};
    if (r < NI) {
      const int ix = r % n, iy = r / n, px = ix + 1, py = iy + 1;
      const double aSW = q4[0], aSE = q4[1], aNW = q4[2], aNE = q4[3];
      fr[0] = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
      constexpr int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
      constexpr int dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
      const double ks[8] = {-(aSW + aNW) * (1.0 / 6.0), -(aSE + aNE) * (1.0 / 6.0), -(aSW + aSE) * (1.0 / 6.0),
                            -(aNW + aNE) * (1.0 / 6.0), -aSW * (1.0 / 3.0),         -aSE * (1.0 / 3.0),
                            -aNW * (1.0 / 3.0),         -aNE * (1.0 / 3.0)};
      constexpr double hinv = 1.0 / M;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int qx = px + dxs[d], qy = py + dys[d];
        const bool bnd = qx == 0 || qx == M || qy == 0 || qy == M;
        const double x = qx * hinv, y = qy * hinv;
        const double k = bnd ? ks[d] : 0.0;
        rhs[0] -= k * ((1.0 - x) * (1.0 - y));
        rhs[1] -= k * (x * (1.0 - y));
        rhs[2] -= k * (x * y);
      }
      // lower interior neighbours: W (offset 1), SE (n-1), S (n), SW (n+1)
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
      for (int l = 0; l < 3; ++l) rhs_out[l] = rhs[l];
    } else {
#pragma unroll
      for (int l = 0; l < 3; ++l) sh.f[r % FW][l] = rhs[l];
    }
  };
  // original values of tile (row tile rt, column tile rt - dt) from sh.fr
  // Couplings sit at three tile offsets: dt = 0 (diagonal and W), dt = 1
  // (the W coupling of the tile's first row, which lies in the previous
  // column tile) and dt = NT-1 (SE and S at the far end of the band).
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
    tile[0][T - 1] = d1 ? sh.fr[0][1] : 0.0;      // offset 1 (W) across the tile edge
    static_assert(T >= 3 && NT >= 3 && T * (NT - 1) == M - T, "band edge inside one tile column");
    tile[T - 2][0] = dl ? sh.fx[0] : 0.0;  // offset n-1 (SE)
    tile[T - 1][1] = dl ? sh.fx[1] : 0.0;
    tile[T - 1][0] = dl ? sh.fx[2] : 0.0;  // offset n (S)
  };

  // ---- initial window: tiles (R, C), R, C < NT, all original ----
  {
    const int R0 = P, C0 = Q;
    double q4[4];
    for (int rt = 0; rt < NT; ++rt) {
      if (g < T) {
        double frv[5];
        load_quad(T * rt + g, q4);
        build_row(T * rt + g, g, q4, frv, nullptr);
      }
      WAVE_SYNC();
      if (R0 == rt) fresh_tile(R0 - C0);
      WAVE_SYNC();
    }
  }

  // prefetch of the coefficients for the rows entering at panel 0
  double q4n[4];
  if (g < T) load_quad(T * NT + g, q4n);

  double ent[3] = {0.0, 0.0, 0.0};  // entering row's right-hand sides (lanes g < T)
  for (int J = 0; J < NP; ++J) {
    const int j0 = J % NT;
    // current tile of this lane: w(X) = J + ((X - J) mod NT)
    const int wP = J + ((P - j0 + NT) % NT), wQ = J + ((Q - j0 + NT) % NT);
    const int R = wP > wQ ? wP : wQ, C = wP > wQ ? wQ : wP;

    // 1. rows entering with row tile J + NT; their panel-column tile
    //    (J+NT, J) has SW, S, SE couplings at columns i, i+1, i+2
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
    // 2. diagonal tile: in-register LDL^T, forward substitution, y y^T / d
    if (R == J && C == J) {
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const double d = tile[k][k];
        bad = bad || !(d > 0.0);
        const double inv = recip(d);
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
      double y[T][3];
#pragma unroll
      for (int k = 0; k < T; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          double v = sh.f[(T * J + k) % FW][l];
#pragma unroll
          for (int kk = 0; kk < k; ++kk) v -= tile[k][kk] * y[kk][l];
          y[k][l] = v;
        }
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const double inv = sh.invd[k];
        const double z0 = y[k][0] * inv, z1 = y[k][1] * inv, z2 = y[k][2] * inv;
        sc[0] += z0 * y[k][0];
        sc[1] += z0 * y[k][1];
        sc[2] += z0 * y[k][2];
        sc[3] += z1 * y[k][1];
        sc[4] += z1 * y[k][2];
        sc[5] += z2 * y[k][2];
        double* fu = sh.f[(T * J + k) % FW];
        fu[0] = z0;
        fu[1] = z1;
        fu[2] = z2;
      }
    } else if (C == J) {
      // 3a. sub-diagonal panel tile (R, J) -> panel rows (R-J-1)*T ...
      const int rb = R - J - 1;
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int k = 0; k < T; ++k) sh.pw[k][rb][i] = tile[i][k];
    }
    WAVE_SYNC();
    // 3b. panel rows: W = A L^{-T}; rhs -= W u.  Rows one at a time (two at
    // a time saves LDS reads of L and u but exceeds the register budget at
    // T = 8).  Lane g < T solves the entering row NE + g last, from and into
    // its registers; the other NE rows go round the lanes (10 t + g), lanes
    // >= T taking the last round.
    {
      constexpr int NR = NT * T, NE = NR - T, RPL = (NR + TL_G - 1) / TL_G;
      static_assert(T * (RPL - 1) + (TL_G - T) * RPL >= NE, "panel rows fit the lanes");
      // the pivot rows' D^{-1} y is the same for every row: read it once
      double ur[T][3];
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const double* fu = sh.f[(T * J + k) % FW];
        ur[k][0] = fu[0];
        ur[k][1] = fu[1];
        ur[k][2] = fu[2];
      }
#pragma unroll 1
      for (int t = 0; t < RPL; ++t) {
        const bool last = t == RPL - 1;
        const bool entering = last && g < T;
        const int rho0 = !last ? TL_G * t + g : (g < T ? NE + g : TL_G * t + g - T);
        const bool ok = entering || rho0 < NE;
        const int rho = ok ? rho0 : 0;
        double w[T], fa[3];
#pragma unroll
        for (int k = 0; k < T; ++k) w[k] = sh.pw[k][rho / T][rho % T];
        {
          const double* fr = sh.f[(T * (J + 1) + rho) % FW];
          fa[0] = entering ? ent[0] : fr[0];
          fa[1] = entering ? ent[1] : fr[1];
          fa[2] = entering ? ent[2] : fr[2];
        }
#pragma unroll
        for (int k = 1; k < T; ++k)
#pragma unroll
          for (int kk = 0; kk < k; ++kk) w[k] -= w[kk] * sh.L[k * (k - 1) / 2 + kk];
#pragma unroll
        for (int k = 0; k < T; ++k) {
          fa[0] -= w[k] * ur[k][0];
          fa[1] -= w[k] * ur[k][1];
          fa[2] -= w[k] * ur[k][2];
        }
        if (ok) {
#pragma unroll
          for (int k = 0; k < T; ++k) sh.pw[k][rho / T][rho % T] = w[k];
          if (entering) {
            ent[0] = fa[0];
            ent[1] = fa[1];
            ent[2] = fa[2];
          } else {
            double* fr = sh.f[(T * (J + 1) + rho) % FW];
            fr[0] = fa[0];
            fr[1] = fa[1];
            fr[2] = fa[2];
          }
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
    WAVE_SYNC();
    // the entering rows' right-hand sides take the retired pivot slots (every
    // read of the pivot rows' D^{-1} y happened before the barrier)
    if (g < T) {
      double* fe = sh.f[(T * (J + NT) + g) % FW];
      fe[0] = ent[0];
      fe[1] = ent[1];
      fe[2] = ent[2];
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
    WAVE_SYNC();
  }

  // ---- g . K_BB g' over the 4(m-1) elements touching the boundary ----
  // (done after the elimination so that these sums are not live across it)
  double sbb[6] = {0, 0, 0, 0, 0, 0};
  for (int e = g; e < 4 * (M - 1); e += TL_G) {
    int ex, ey;
    if (e < M) { ex = e; ey = 0; }                         // bottom row
    else if (e < 2 * M) { ex = e - M; ey = M - 1; }        // top row
    else if (e < 3 * M - 2) { ex = 0; ey = e - 2 * M + 1; } // left column, corners excluded
    else { ex = M - 1; ey = e - (3 * M - 2) + 1; }         // right column, corners excluded
    const double ae = ld(a, ey * lda + ex);
    int qq = 0;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int lp = l; lp < 3; ++lp) sbb[qq++] += ae * bb_coef(l, lp, ex, ey, M);
  }

  // ---- reduce the ten lanes' partial energies and write S ----
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    sh.red[g][t] = sbb[t];
    sh.red[g][6 + t] = sc[t];
  }
  sh.red[g][12] = bad ? 1.0 : 0.0;
  WAVE_SYNC();
  if (g == 0 && valid) {
    double t6[6];
    bool anybad = false;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      double b = 0.0, c = 0.0;
      for (int h = 0; h < TL_G; ++h) {
        b += sh.red[h][t];
        c += sh.red[h][6 + t];
      }
      t6[t] = b - c;
    }
    for (int h = 0; h < TL_G; ++h) anybad = anybad || sh.red[h][12] != 0.0;
    const double s3[3][3] = {{t6[0], t6[1], t6[2]}, {t6[1], t6[3], t6[4]}, {t6[2], t6[4], t6[5]}};
    store_packed(args.S + p * 10, s3);
    if (args.status) args.status[p] = anybad ? STOMSFEM_ENOTSPD : STOMSFEM_OK;
  }
}

template <int M, int T, typename TA, int WV>
// Occupancy floor: at m = 16 four wavefronts per SIMD (the LDS limit) beat
// the spill-free register allocation (two) by 40% even with spills; at m = 32
// two wavefronts per SIMD without spills.
__global__ __launch_bounds__(64 * WV, (M == 16 ? 4 : 2)) void upscale_tiled_kernel(UpArgs args) {
  __shared__ TiledLds<M, T> lds_all[WV][TL_SLOTS];
  // WV independent wavefronts per workgroup (a launch-shape choice only)
  const int wave = threadIdx.x >> 6;
  tiled_wave<M, T, TA>(args, (int64_t)blockIdx.x * WV + wave, threadIdx.x & 63, lds_all[wave]);
}

bool tiled_supports(int m) { return m == 16 || m == 32; }

template <int M, int T, int WV>
static hipError_t launch_t(const UpArgs& args, int a_dtype, hipStream_t st) {
  const int64_t per_block = (int64_t)TL_SLOTS * WV;
  const int64_t blocks = (args.npairs + per_block - 1) / per_block;
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL((upscale_tiled_kernel<M, T, float, WV>), dim3((unsigned)blocks), dim3(64 * WV), 0, st, args);
  else
    hipLaunchKernelGGL((upscale_tiled_kernel<M, T, double, WV>), dim3((unsigned)blocks), dim3(64 * WV), 0, st, args);
  return hipGetLastError();
}

template <int M, int T>
static hipError_t launch_tw(const UpArgs& args, int a_dtype, hipStream_t st, int waves) {
  if (waves == 2) return launch_t<M, T, 2>(args, a_dtype, st);
  return launch_t<M, T, 1>(args, a_dtype, st);
}

hipError_t launch_upscale_tiled(const UpArgs& args, int a_dtype, hipStream_t st, int waves) {
  if (args.m == 16) return launch_tw<16, 4>(args, a_dtype, st, waves);
  if (args.m == 32) return launch_tw<32, 8>(args, a_dtype, st, waves);
  return hipErrorInvalidValue;
}

// ---- one persistent launch over batches of several m (8, 16, 32) ----
//
// A single queue of work items spans every batch; each wavefront takes the
// next item with one atomic increment and loops until the queue is empty.  An
// item is one wavefront's tile: TL_SLOTS pairs for m = 16 and 32 (the
// register-tiled elimination above), 64 pairs for m = 8 (one pair per lane,
// small_cell.h).  Items are numbered by decreasing cost -- every m = 32 item
// first, then m = 16, then m = 8 -- so the costliest items are taken first and
// the launch ends on the cheapest ones (longest-processing-time-first list
// scheduling on the CUs).  Every pair runs the same device code as in the
// per-m kernels, so S and the status are bitwise those of stomsfem_upscale.
// Registers and LDS are the maximum over the three paths: two wavefronts per
// SIMD, the m = 32 limits (m = 16 tiles run at half their own kernel's
// occupancy, m = 8 lanes at their register limit).
struct QueueBatch {
  UpArgs args;
  int64_t first;  // number of the batch's first item
  int32_t m;
};
constexpr int QUEUE_MAXB = 8;
struct QueueArgs {
  QueueBatch b[QUEUE_MAXB];  // in item order: m = 32, then 16, then 8
  int32_t nb;
  int64_t total;             // items in all
  unsigned long long* counter;
};

__global__ void queue_reset_kernel(unsigned long long* counter) {
  if (threadIdx.x == 0) *counter = 0ull;
}

template <typename TA>
__global__ __launch_bounds__(128, 2) void upscale_queue_kernel(QueueArgs qa) {
  // one union per wavefront, so that each wavefront's blocks stay its own
  // whichever m its current item has
  union WaveLds {
    TiledLds<32, 8> l32[TL_SLOTS];
    TiledLds<16, 4> l16[TL_SLOTS];
  };
  __shared__ WaveLds lds[2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (;;) {
    unsigned long long it = 0;
    if (lane == 0) it = atomicAdd(qa.counter, 1ull);
    // the item number is wavefront-uniform: keep it (and what follows from
    // it) in scalar registers
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)it);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(it >> 32));
    const int64_t item = (int64_t)(((uint64_t)hi << 32) | lo);
    if (item >= qa.total) break;
    int b = 0;
    while (b + 1 < qa.nb && item >= qa.b[b + 1].first) ++b;
    const UpArgs args = qa.b[b].args;
    const int64_t local = item - qa.b[b].first;
    const int m = qa.b[b].m;
    if (m == 32) {
      tiled_wave<32, 8, TA>(args, local, lane, lds[wave].l32);
    } else if (m == 16) {
      tiled_wave<16, 4, TA>(args, local, lane, lds[wave].l16);
    } else {
      const int64_t p = local * 64 + lane;
      if (p < args.npairs) {
        const int Mc = args.ncx * args.ncy;
        const int64_t s = p / Mc;
        const int K = (int)(p - s * Mc);
        small_cell_solve<8, TA>((const TA*)args.a + block_offset(s, K, args.ncx, args.ncy, 8),
                                (int64_t)args.ncx * 8, args.S + p * 10, args.status ? args.status + p : nullptr);
      }
    }
  }
}

bool queue_supports(int m) { return m == 8 || m == 16 || m == 32; }
int queue_max_batches() { return QUEUE_MAXB; }

// batches: nb <= QUEUE_MAXB, every m in {8, 16, 32}, one coefficient type;
// counter: 8 bytes of device memory, reset here on the stream.
hipError_t launch_upscale_queue(const UpArgs* batches, int nb, int a_dtype, unsigned long long* counter,
                                hipStream_t st) {
  if (nb < 1 || nb > QUEUE_MAXB) return hipErrorInvalidValue;
  QueueArgs qa{};
  int64_t total = 0;
  for (int mm : {32, 16, 8}) {
    for (int i = 0; i < nb; ++i) {
      if (!queue_supports(batches[i].m)) return hipErrorInvalidValue;
      if (batches[i].m != mm || batches[i].npairs == 0) continue;
      QueueBatch& q = qa.b[qa.nb++];
      q.args = batches[i];
      q.first = total;
      q.m = mm;
      const int64_t per = mm == 8 ? 64 : TL_SLOTS;
      total += (batches[i].npairs + per - 1) / per;
    }
  }
  if (total == 0) return hipSuccess;
  qa.total = total;
  qa.counter = counter;
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = a_dtype == STOMSFEM_F32
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, upscale_queue_kernel<float>, 128, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, upscale_queue_kernel<double>, 128, 0);
  if (e != hipSuccess) return e;
  int64_t grid = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
  const int64_t waves_needed = (total + 1) / 2;  // two wavefronts per workgroup
  if (grid > waves_needed) grid = waves_needed;
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, counter);
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(upscale_queue_kernel<float>, dim3((unsigned)grid), dim3(128), 0, st, qa);
  else
    hipLaunchKernelGGL(upscale_queue_kernel<double>, dim3((unsigned)grid), dim3(128), 0, st, qa);
  return hipGetLastError();
}

}  // namespace stomsfem
