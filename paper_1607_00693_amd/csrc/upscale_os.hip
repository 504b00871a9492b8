// Oversampled local upscaling with the Petrov-Galerkin stiffness (Sec. 2.2,
// remark on oversampling; eq. stiffness_local_petrov).
//
// For the coarse element K the cell problems (eq. MsFEB) are solved on a
// patch of M = m + 2o fine cells per side around K (moved inside the domain
// at its edges), with the bilinear nodal functions g^j of the patch corners
// as boundary data: psi^j, j = 0..3, psi^3 = 1 - psi^0 - psi^1 - psi^2.  All
// the Petrov-Galerkin stiffness needs of them is linear in psi^j, so it comes
// out of the same sliding-window LDL^T as the plain path, with test vectors
// carried through the forward substitution beside the three data sets
// f^j = -K_IB g^j:
//   psi^j(x_k) = e_k . K_II^{-1} f^j          (corner x_k of K inside the patch)
//   A[j][l]    = psi^j . r^l,  r^l = K^K p^l  (K^K: fine stiffness of K's
//                elements; p^l: K's bilinear nodal functions)
// and, with K_II = L D L^T, u . K_II^{-1} v = sum_k (L^{-1}u)_k (L^{-1}v)_k / d_k.
// C = Psi^{-T} makes phi^i = sum_j C[i][j] psi^j nodal at K's corners, and
// S[l][l'] = int_K a grad phi^l . grad p^l' = (C A)[l][l'].
//
// One wavefront per pair: the (M+1) x (M+1) circular band window and the ten
// right-hand-side columns live in LDS (with the lifts, 14.6 KB at M = 32; 39 KB
// at M = 64, so several pairs share a CU); the patch coefficients stay in
// global memory, the four around the next entering row's node are fetched a
// pivot ahead, and the entering row and its r^l are formed from them; the
// rank-1 update of each pivot is spread over the 64 lanes; no workgroup
// barriers.
#include "common.h"

namespace stomsfem {

#define OS_WAVE_SYNC()                                     \
  do {                                                     \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                       \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
  } while (0)

constexpr int OS_NV = 10;    // columns: f^0..2, corner tests 0..3, r^0..2
constexpr int OS_MAXM = 64;  // largest patch (band half-width); 64-cell patches need 104 KB of LDS
constexpr int OS_EP = 32;    // epilogue scratch per wavefront (doubles)

struct OsArgs {
  UpArgs up;  // up.m = m; up.S = S16 output [npairs][16]
  int32_t o;  // fine cells added on each side of K
  // optional: solve only the pairs list[i], i < nlist, into S[i], status[i]
  const int64_t* list;
  int64_t nlist;
};

// first fine cell (one axis) of the patch of coarse element k
__host__ __device__ inline int os_origin(int k, int m, int o, int nf) {
  int x0 = k * m - o;
  if (x0 > nf - (m + 2 * o)) x0 = nf - (m + 2 * o);
  return x0 < 0 ? 0 : x0;
}

// Patches of up to OS_TABM cells (the kernels with at most 9 trailing entries
// per lane) keep the lifts of the rows next to the patch boundary in LDS,
// formed once per pair (3 KB at 32 cells), and form r^l of an entering row in
// closed form (os_rK_cf): the kernel then stays within 128 registers (four
// wavefronts per SIMD) and 14.6 KB of LDS per pair at 32 cells (ten pairs
// per CU).  Larger patches form both on the fly with the general os_rK.
constexpr int OS_TABM = 33;
__host__ __device__ inline bool os_tables(int M) { return M <= OS_TABM; }
__host__ __device__ inline int os_lds_doubles(int, int M) {
  const int WN = M + 1;
  return WN * WN + WN * OS_NV + OS_EP + (os_tables(M) ? 3 * 4 * M : 0);
}

// x mod w for 0 <= x < 2w
__device__ __forceinline__ int os_wrap(int x, int w) { return x >= w ? x - w : x; }

// Bilinear corner function p^l (l = 0..2) at node (px, py) of a grid with
// 1/size = rs (a multiplication where pcorner divides: equal for powers of
// two, within an ulp otherwise).
__device__ __forceinline__ double os_pc(int l, int px, int py, double rs) {
  const double x = px * rs, y = py * rs;
  return l == 0 ? (1.0 - x) * (1.0 - y) : l == 1 ? x * (1.0 - y) : x * y;
}

// r^l = (K^K p^l) at patch node (px, py): the elements of K around the node
// (SW, SE, NW, NE see it as local node 2, 3, 1, 0), each a_e K_ref p^l_e;
// q4 = the coefficients of the four elements around the node (SW, SE, NW, NE).
__device__ inline double os_rK(int l, int px, int py, int cx, int cy, int m, const double* q4) {
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
      s += kref(al, be) * os_pc(l, bx - cx, by - cy, rm);
    }
    v += q4[e] * s;
  }
  return v;
}

// The same r^l in closed form.  On element e of K at (xe, ye) = its lower-left
// node relative to K's, p^l is bilinear in the element's local coordinates
// (s, t): A + B s + C t + D s t with (times m^2)
//   l = 0: B = -(m - ye), C = -(m - xe), D = 1;
//   l = 1: B =  (m - ye), C = -xe,       D = -1;
//   l = 2: B =  ye,       C = xe,        D = 1,
// and K_ref annihilates constants, so row al of K_ref applied to its corner
// values is B sig_s(al) + C sig_t(al) + D sig_st(al), with sig_s = K_ref row
// sums over the corners with s = 1, sig_t over t = 1, sig_st over s = t = 1:
// (-1/2, -1/2, -1/3), (1/2, -1/2, -1/6), (1/2, 1/2, 2/3), (-1/2, 1/2, -1/6)
// for al = 0..3.
__device__ inline double os_rK_cf(int l, int px, int py, int cx, int cy, int m, const double* q4) {
  const double im2 = 1.0 / ((double)m * m);
  double v = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ex = px - 1 + (e & 1), ey = py - 1 + (e >> 1);
    if (ex < cx || ex >= cx + m || ey < cy || ey >= cy + m) continue;
    const double xe = ex - cx, ye = ey - cy;
    // local index of the node in element e: SW -> 2, SE -> 3, NW -> 1, NE -> 0
    const double ss = (e == 0 || e == 2) ? 0.5 : -0.5;            // al = 2, 1 : 1/2; al = 3, 0 : -1/2
    const double st = (e == 0 || e == 1) ? 0.5 : -0.5;            // al = 2, 3 : 1/2; al = 1, 0 : -1/2
    const double sst = e == 0 ? 2.0 / 3.0 : (e == 3 ? -1.0 / 3.0 : -1.0 / 6.0);
    double B, C, D;
    if (l == 0) {
      B = -(m - ye);
      C = -(m - xe);
      D = 1.0;
    } else if (l == 1) {
      B = m - ye;
      C = -xe;
      D = -1.0;
    } else {
      B = ye;
      C = xe;
      D = 1.0;
    }
    v += q4[e] * ((B * ss + C * st + D * sst) * im2);
  }
  return v;
}

// NQ >= B (B + 1) / (2 * 64): trailing-triangle entries per lane.
template <typename TA, int NQ>
__global__ __launch_bounds__(256) void upscale_os_kernel(OsArgs args) {
  extern __shared__ double smem[];
  const int m = args.up.m, o = args.o, M = m + 2 * o, n = M - 1, NI = n * n, B = M, WN = B + 1;
  const int waves = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* Wn = smem + wave * os_lds_doubles(m, M);  // window, (r, c) at [r % WN][c % WN]
  double* R = Wn + WN * WN;                          // right-hand sides, row r at [r % WN][OS_NV]
  double* Ep = R + WN * OS_NV;                       // epilogue scratch
  constexpr bool tab = NQ <= 9;  // with M <= 33 exactly (os_tables)
  double* Fb = Ep + OS_EP;                           // lifts of the rows next to the boundary [ring][3] (tab)
  const int64_t io = (int64_t)blockIdx.x * waves + wave;  // output slot
  if (io >= (args.list ? args.nlist : args.up.npairs)) return;  // the whole wavefront; no workgroup barrier follows
  const int64_t p = args.list ? args.list[io] : io;
  const int ncx = args.up.ncx, ncy = args.up.ncy, Mc = ncx * ncy;
  const int64_t s = p / Mc;
  const int K = (int)(p - s * Mc), kx = K % ncx, ky = K / ncx;
  const int nfx = ncx * m, nfy = ncy * m;
  const int x0 = os_origin(kx, m, o, nfx), y0 = os_origin(ky, m, o, nfy);
  const int cx = kx * m - x0, cy = ky * m - y0;  // K's lower-left node in patch nodes
  const TA* a = (const TA*)args.up.a + s * (int64_t)nfy * nfx + (int64_t)y0 * nfx + x0;  // patch origin
  for (int i = lane; i < WN * WN; i += 64) Wn[i] = 0.0;
  for (int i = lane; i < WN * OS_NV; i += 64) R[i] = 0.0;
  OS_WAVE_SYNC();
  const double rM = 1.0 / M;
  // coefficients of the four patch elements around interior node (ix, iy):
  // SW, SE, NW, NE (every lane loads the same four values)
  auto load_quad = [&](int ix, int iy, double* q4) {
    q4[0] = ld(a, (int64_t)iy * nfx + ix);
    q4[1] = ld(a, (int64_t)iy * nfx + ix + 1);
    q4[2] = ld(a, (int64_t)(iy + 1) * nfx + ix);
    q4[3] = ld(a, (int64_t)(iy + 1) * nfx + ix + 1);
  };
  // f^v = -sum over the boundary neighbours q of K[r][q] g^v(q), for the row
  // of interior node (ix, iy) with coefficients q4
  auto lift = [&](int v, int ix, int iy, const double* q4) {
    const int px = ix + 1, py = iy + 1;
    const double aSW = q4[0], aSE = q4[1], aNW = q4[2], aNE = q4[3];
    const int dxs[8] = {-1, 1, 0, 0, -1, 1, -1, 1};
    const int dys[8] = {0, 0, -1, 1, -1, -1, 1, 1};
    const double ks[8] = {-(aSW + aNW) * (1.0 / 6.0), -(aSE + aNE) * (1.0 / 6.0), -(aSW + aSE) * (1.0 / 6.0),
                          -(aNW + aNE) * (1.0 / 6.0), -aSW * (1.0 / 3.0),         -aSE * (1.0 / 3.0),
                          -aNW * (1.0 / 3.0),         -aNE * (1.0 / 3.0)};
    double val = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int qx = px + dxs[q], qy = py + dys[q];
      if (qx == 0 || qx == M || qy == 0 || qy == M) val -= ks[q] * os_pc(v, qx, qy, rM);
    }
    return val;
  };
  // coefficients of the patch elements around node (ax, ay), 0 outside the
  // patch (os_rK reads only elements of K)
  auto quad_at = [&](int ax, int ay, double* q4) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ex = ax - 1 + (e & 1), ey = ay - 1 + (e >> 1);
      q4[e] = (ex >= 0 && ex < M && ey >= 0 && ey < M) ? ld(a, (int64_t)ey * nfx + ex) : 0.0;
    }
  };
  // ring position of an interior node next to the boundary: bottom, right,
  // top, left (corners once)
  const int nring = n == 1 ? 1 : 4 * (n - 1);
  auto ring_pos = [&](int ix, int iy) {
    if (n == 1) return 0;
    if (iy == 0) return ix;
    if (ix == n - 1) return (n - 1) + iy;
    if (iy == n - 1) return 2 * (n - 1) + (n - 1 - ix);
    return 3 * (n - 1) + (n - 1 - iy);
  };
  if constexpr (tab) {
    for (int i = lane; i < 3 * nring; i += 64) {
      const int v = i / nring, b = i - v * nring;
      int ix, iy;
      if (n == 1) { ix = 0; iy = 0; }
      else if (b < n - 1) { ix = b; iy = 0; }
      else if (b < 2 * (n - 1)) { ix = n - 1; iy = b - (n - 1); }
      else if (b < 3 * (n - 1)) { ix = n - 1 - (b - 2 * (n - 1)); iy = n - 1; }
      else { ix = 0; iy = n - 1 - (b - 3 * (n - 1)); }
      double q4[4];
      load_quad(ix, iy, q4);
      Fb[b * 3 + v] = lift(v, ix, iy, q4);
    }
  }
  // this lane's entries (io >= ko) of the B x B trailing triangle
  int tik[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = lane + 64 * q;
    int io = 0;
    while ((io + 1) * (io + 2) / 2 <= t) ++io;
    tik[q] = t < B * (B + 1) / 2 ? (io | ((t - io * (io + 1) / 2) << 8)) : B;
  }
  OS_WAVE_SYNC();

  // original row r = iy n + ix of K_II, in window slot rs (slots 0..B: band
  // entry at distance u; B+1..B+OS_NV: its ten right-hand sides), from the
  // coefficients q4 of the four elements around its node
  auto insert_row = [&](int r, int rs, int ix, int iy, const double* q4) {
    const int px = ix + 1, py = iy + 1;
    // wave-uniform: only rows next to the patch boundary have lifts, only
    // nodes of K carry r^l
    const bool nearb = ix == 0 || ix == n - 1 || iy == 0 || iy == n - 1;
    const bool inK = px >= cx && px <= cx + m && py >= cy && py <= cy + m;
    const double aSW = q4[0], aSE = q4[1], aNW = q4[2], aNE = q4[3];
    // slots u = 0..B: band entry at distance u; u = B+1..B+OS_NV: the ten
    // right-hand sides (two rounds of the wavefront when B + OS_NV >= 64)
    for (int u = lane; u <= B + OS_NV; u += 64) {
      if (u <= B) {
        const int t = u;
        double v = 0.0;
        if (t == 0) v += (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
        if (t == 1 && ix >= 1) v += -(aSW + aNW) * (1.0 / 6.0);
        if (t == n - 1 && iy >= 1 && ix <= n - 2) v += -aSE * (1.0 / 3.0);
        if (t == n && iy >= 1) v += -(aSW + aSE) * (1.0 / 6.0);
        if (t == n + 1 && iy >= 1 && ix >= 1) v += -aSW * (1.0 / 3.0);
        if (r - t >= 0) Wn[rs * WN + (rs - t >= 0 ? rs - t : rs - t + WN)] = v;
      } else {
        const int v = u - B - 1;
        double val = 0.0;
        if (v < 3) {
          if (nearb) {
            if constexpr (tab) val = Fb[ring_pos(ix, iy) * 3 + v];
            else val = lift(v, ix, iy, q4);
          }
        } else if (v < 7) {
          const int k = v - 3;  // corner k of K (CCW from lower left)
          const int kpx = cx + ((k == 1 || k == 2) ? m : 0), kpy = cy + (k >= 2 ? m : 0);
          val = (px == kpx && py == kpy) ? 1.0 : 0.0;
        } else if (inK) {
          if constexpr (tab) val = os_rK_cf(v - 7, px, py, cx, cy, m, q4);
          else val = os_rK(v - 7, px, py, cx, cy, m, q4);
        }
        R[rs * OS_NV + v] = val;
      }
    }
  };

  const int r0 = B < NI ? B : NI;
  for (int r = 0; r < r0; ++r) {
    double q4[4];
    load_quad(r % n, r / n, q4);
    insert_row(r, r, r % n, r / n, q4);
  }
  OS_WAVE_SYNC();
  // the row entering at pivot j is j + B: slot (j + B) mod WN = (j - 1) mod WN,
  // node (eix, eiy), both advanced incrementally
  int eix = B % n, eiy = B / n;
  double q4n[4] = {0.0, 0.0, 0.0, 0.0};  // the next entering row's coefficients, fetched a pivot ahead
  if (B < NI) load_quad(eix, eiy, q4n);
  // lanes 0..20 accumulate Y[jv][tv] = f^jv . K_II^{-1} (test column 3 + tv)
  const int jv = lane / 7, tv = 3 + lane % 7;
  double yacc = 0.0;
  bool bad = false;
  for (int j = 0, jj = 0; j < NI; ++j, jj = jj + 1 == WN ? 0 : jj + 1) {
    if (j + B < NI) {
      const double q4[4] = {q4n[0], q4n[1], q4n[2], q4n[3]};
      int nix = eix + 1, niy = eiy;
      if (nix == n) {
        nix = 0;
        ++niy;
      }
      if (j + B + 1 < NI) load_quad(nix, niy, q4n);
      insert_row(j + B, jj == 0 ? WN - 1 : jj - 1, eix, eiy, q4);
      OS_WAVE_SYNC();
      eix = nix;
      eiy = niy;
    }
    const double d = Wn[jj * WN + jj];
    bad = bad || !(d > 0.0);
    // 1/d from the hardware estimate and two Newton steps (full FP64 accuracy)
    double inv = __builtin_amdgcn_rcp(d);
    inv = __builtin_fma(inv, __builtin_fma(-d, inv, 1.0), inv);
    inv = __builtin_fma(inv, __builtin_fma(-d, inv, 1.0), inv);
    const int cnt = (j + B < NI - 1 ? j + B : NI - 1) - j;
    if (lane < 21) yacc += R[jj * OS_NV + jv] * R[jj * OS_NV + tv] * inv;
    double wv[NQ];
    int idx[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int io = tik[q] & 255, ko = tik[q] >> 8;
      const int ri = os_wrap(jj + 1 + io, WN), rk = os_wrap(jj + 1 + ko, WN);
      idx[q] = ri * WN + rk;
      wv[q] = io < cnt ? Wn[idx[q]] - Wn[ri * WN + jj] * inv * Wn[rk * WN + jj] : 0.0;
    }
    for (int e = lane; e < cnt * OS_NV; e += 64) {
      const int t = 1 + e / OS_NV, v = e - (t - 1) * OS_NV;
      const int rt = os_wrap(jj + t, WN);
      R[rt * OS_NV + v] -= Wn[rt * WN + jj] * inv * R[jj * OS_NV + v];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if ((tik[q] & 255) < cnt) Wn[idx[q]] = wv[q];
    OS_WAVE_SYNC();
  }

  // g^j . r^l over K's nodes on the patch boundary (K touches it only at the
  // edges of the domain, where the patch is moved inside)
  double bt[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) bt[q] = 0.0;
  for (int id = lane; id < (m + 1) * (m + 1); id += 64) {
    const int ax = cx + id % (m + 1), ay = cy + id / (m + 1);
    if (!(ax == 0 || ax == M || ay == 0 || ay == M)) continue;
    double q4[4];
    quad_at(ax, ay, q4);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double rl = os_rK(l, ax, ay, cx, cy, m, q4);
#pragma unroll
      for (int jb = 0; jb < 3; ++jb) bt[3 * jb + l] += os_pc(jb, ax, ay, rM) * rl;
    }
  }
#pragma unroll
  for (int q = 0; q < 9; ++q)
    for (int off = 32; off > 0; off >>= 1) bt[q] += __shfl_xor(bt[q], off, 64);
  if (lane < 21) Ep[lane] = yacc;
  OS_WAVE_SYNC();
  if (lane == 0) {
    // Psi[k][j] = psi^j(x_k); corners on the patch boundary carry the data
    double Psi[4][4], A[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int kpx = cx + ((k == 1 || k == 2) ? m : 0), kpy = cy + (k >= 2 ? m : 0);
      const bool onb = kpx == 0 || kpx == M || kpy == 0 || kpy == M;
      double sum = 0.0;
#pragma unroll
      for (int jb = 0; jb < 3; ++jb) {
        Psi[k][jb] = onb ? os_pc(jb, kpx, kpy, rM) : Ep[jb * 7 + k];
        sum += Psi[k][jb];
      }
      Psi[k][3] = 1.0 - sum;
    }
    // A[j][l] = int_K a grad psi^j . grad p^l; row and column 3 from the
    // partitions of unity of psi and p
#pragma unroll
    for (int jb = 0; jb < 3; ++jb) {
      double rs = 0.0;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        A[jb][l] = bt[3 * jb + l] + Ep[jb * 7 + 4 + l];
        rs += A[jb][l];
      }
      A[jb][3] = -rs;
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) A[3][l] = -(A[0][l] + A[1][l] + A[2][l]);
    // C = (Psi^T)^{-1}: Gauss-Jordan with partial pivoting on [Psi^T | I]
    double G[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 8; ++c) G[i][c] = c < 4 ? Psi[c][i] : (c - 4 == i ? 1.0 : 0.0);
    // (every index compile-time: the row interchange is a select per entry)
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
    if (args.up.status) args.up.status[io] = (bad || sing) ? STOMSFEM_ENOTSPD : STOMSFEM_OK;
  }
}

size_t upscale_os_lds_bytes(int m, int o, int waves) {
  return sizeof(double) * (size_t)os_lds_doubles(m, m + 2 * o) * waves;
}

// wavefronts (pairs) per workgroup: within 64 KB of LDS, the count that puts
// the most wavefronts on a CU's 160 KB (the larger one on a tie)
int upscale_os_waves(int m, int o) {
  int best = 1;
  size_t best_waves = 0;
  for (int w = 1; w <= 4; ++w) {
    const size_t b = upscale_os_lds_bytes(m, o, w);
    if (b > 64 * 1024) break;
    const size_t on_cu = (160 * 1024 / b) * w;
    if (on_cu >= best_waves) {
      best_waves = on_cu;
      best = w;
    }
  }
  return best;
}

bool upscale_os_supports(int m, int o) { return m >= 1 && o >= 0 && m + 2 * o >= 2 && m + 2 * o <= OS_MAXM; }

// Launch with `lds` bytes of dynamic LDS; above 64 KB the kernel's limit is
// raised first (a host call before each such launch, so it holds on whichever
// device is current).
template <typename TA, int NQ>
static hipError_t launch_os_nq(const OsArgs& args, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)upscale_os_kernel<TA, NQ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((upscale_os_kernel<TA, NQ>), grid, block, lds, st, args);
  return hipGetLastError();
}

template <typename TA>
static hipError_t launch_os_t(const OsArgs& args, hipStream_t st) {
  const int M = args.up.m + 2 * args.o;
  const int waves = upscale_os_waves(args.up.m, args.o);
  const int64_t blocks = ((args.list ? args.nlist : args.up.npairs) + waves - 1) / waves;
  const size_t lds = upscale_os_lds_bytes(args.up.m, args.o, waves);
  const int need = (M * (M + 1) / 2 + 63) / 64;
  const dim3 grid((unsigned)blocks), block(64 * waves);
  if (need <= 3) return launch_os_nq<TA, 3>(args, grid, block, lds, st);
  if (need <= 5) return launch_os_nq<TA, 5>(args, grid, block, lds, st);
  if (need <= 9) return launch_os_nq<TA, 9>(args, grid, block, lds, st);
  if (need <= 17) return launch_os_nq<TA, 17>(args, grid, block, lds, st);
  return launch_os_nq<TA, 33>(args, grid, block, lds, st);
}

bool upscale_os_tiled_supports(int m, int o);
hipError_t launch_upscale_os_tiled(const UpArgs& up, int o, int a_dtype, hipStream_t st, const int64_t* list,
                                   int64_t nlist);

// list != nullptr: only the pairs list[i] (i < nlist) of the batch, their
// S and status written compactly at i.
hipError_t launch_upscale_os(const UpArgs& up, int o, int a_dtype, hipStream_t st, const int64_t* list,
                             int64_t nlist) {
  if (!upscale_os_supports(up.m, o)) return hipErrorInvalidValue;
  if ((list ? nlist : up.npairs) <= 0) return hipSuccess;
  // 16- and 24-cell patches: the register-tiled kernel (six pairs per wavefront)
  if (upscale_os_tiled_supports(up.m, o)) return launch_upscale_os_tiled(up, o, a_dtype, st, list, nlist);
  const OsArgs args{up, o, list, nlist};
  return a_dtype == STOMSFEM_F32 ? launch_os_t<float>(args, st) : launch_os_t<double>(args, st);
}

}  // namespace stomsfem
