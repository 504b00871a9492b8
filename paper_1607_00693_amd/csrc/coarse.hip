// Batched coarse solve S U = b (Sec. 2.2 eq. upscaleSUF) with the
// Petrov-Galerkin load (eq. stiffness_local_petrov), and the Monte Carlo
// mean / variance of the coarse solution (Sec. 4.1.1).
//
// One workgroup per sample.  The interior coarse nodes in natural order give
// a 9-point band of half-width ncx; the global stiffness rows are assembled
// on the fly from the four upscaled element matrices around each node as
// they enter an LDS window of (ncx+1) x (ncx+1) entries.
//
// Forward pass: FP64 LDL^T with the forward substitution fused, one
// workgroup barrier per pivot column.  In the phase of pivot j every thread
// applies the rank-1 update of pivot j to its fixed entries of the trailing
// triangle; the threads whose entries make up column j+1 also write it (and
// 1/d_{j+1}) to the other half of a double-buffered LDS column, so pivot j+1
// can start right after the barrier.  The same phase does the forward
// substitution step of pivot j, writes column j of L to a per-workgroup
// slice of the library workspace and assembles the row entering the window
// (its coefficients and load prefetched into registers a phase or a node row
// ahead, so no global load sits between two barriers).
//
// Backward pass L^T x = z, z = D^{-1} y (column-oriented, a second kernel
// with one wavefront per sample, so that the forward kernel keeps its small
// register footprint and the backward passes of many samples overlap):
// lane l keeps z_i for the indices i = l (mod 64) of three consecutive blocks
// of 64 unknowns in registers.  Step j reads x_j = z_j from lane j mod 64 (a
// cross-lane read, no memory round trip) and subtracts l_{j,i} x_j from the
// z_i, i in [j-B, j), of every lane; the L entries are loaded a few steps
// ahead, and the z values of the block after next one block ahead.
#include "common.h"

namespace stomsfem {

constexpr int COARSE_THREADS = 1024;
constexpr int COARSE_NQ = 3;  // largest NQ: B (B+1)/2 <= 3072
constexpr int COARSE_BMAX = 72;
constexpr int COARSE_PG_BMAX = 64;
constexpr int COARSE_SMALL_B = 32;  // largest band served by the one-wavefront workgroup  // Petrov-Galerkin: full B x B trailing square, <= 16 entries per lane
constexpr int COARSE_PD = 32;  // backward substitution: L entries loaded this many steps ahead

// Workgroup barrier that orders LDS only: a pivot step does not wait for
// its global stores (retired L columns, y_j) to complete.
#define COARSE_SYNC()                                                 \
  do {                                                                \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");   \
    __builtin_amdgcn_s_barrier();                                     \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");   \
  } while (0)

// x mod w for 0 <= x < 2w
__device__ __forceinline__ int wrap(int x, int w) { return x >= w ? x - w : x; }

// value of v in lane `lane` (wave-uniform lane index)
__device__ __forceinline__ double lane_value(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

struct CoarseArgs {
  int32_t ncx, ncy;
  int64_t nsamples;
  const double* S;
  const double* load;
  double* U;
  int32_t* status;
  double* work;  // nsamples * (nU * (ncx+1) + 1) doubles (one launch's samples)
};

// Entry of an element matrix with trial index tr and test index te: the
// packed symmetric form, or the 16 row-major entries S[trial][test] of the
// Petrov-Galerkin local stiffness (eq. stiffness_local_petrov).
template <bool PG>
__device__ __forceinline__ double sget(const double* Sk, int tr, int te);

__device__ __forceinline__ double selem(const double* Sk, int i, int j) {
  // packed upper triangle 00,01,02,03,11,12,13,22,23,33
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
  const int base = i == 0 ? 0 : i == 1 ? 4 : i == 2 ? 7 : 9;
  return Sk[base + (j - i)];
}

template <>
__device__ __forceinline__ double sget<false>(const double* Sk, int tr, int te) {
  return selem(Sk, tr, te);
}
template <>
__device__ __forceinline__ double sget<true>(const double* Sk, int tr, int te) {
  return Sk[4 * tr + te];
}

// L entries of backward step j for lane `lam`, zero where the lane's index is
// not in [j-B, j).  Lc column i: [1/d_i, l_{i+1,i}, ..., l_{i+B,i}], so
// l_{j,i} = Lc[i WN + j - i]; for the lane's index i = 64 k' + lam of block
// k' that is Lc[(64 k' + lam)(WN - 1) + j].  Lanes outside the band read the
// zero kept at Lc[zero], so that the loaded value is used as is and the load
// is waited for only where it is consumed, COARSE_PD steps later.
struct BackStep {
  double lc, l1, l2;
};

// FAR: B may exceed 64, so indices two blocks down can be in [j-B, j)
template <bool FAR>
__device__ __forceinline__ BackStep back_loads(const double* Lc, int64_t zero, int WN, int B, int nU, int j,
                                               int lam) {
  // every step issues the same loads (out-of-range steps read the zero), so
  // that the number of loads in flight behind any one of them is fixed
  BackStep r{0.0, 0.0, 0.0};
  const bool in = j >= 0 && j < nU;
  const int k = j >> 6, u = j & 63;
  const int dc = u - lam;  // offset j - i in block k; + 64 in block k-1, + 128 in block k-2
  const bool oc = in && dc >= 1 && dc <= B, o1 = in && k >= 1 && dc + 64 <= B;
  const int64_t base = (int64_t)(64 * k + lam) * (WN - 1) + j;  // block k
  const int64_t step = (int64_t)64 * (WN - 1);
  r.lc = Lc[oc ? base : zero];
  r.l1 = Lc[o1 ? base - step : zero];
  if (FAR) {
    const bool o2 = in && k >= 2 && dc + 128 <= B;
    r.l2 = Lc[o2 ? base - 2 * step : zero];
  }
  return r;
}

// NQ = trailing entries per lane: >= B (B+1) / (2 * 256) for the symmetric
// triangle (NQ = 4 serves B <= 44), >= B^2 / 256 for the Petrov-Galerkin
// square.  PG: element matrices of 16 entries S[trial][test], the coarse
// matrix G[test node][trial node] is non-symmetric and is factored G = L U
// without pivoting (the pivot row goes to the next phase beside the pivot
// column; the backward pass solves U x = y in the form x = z - (D^{-1} U - I) x
// with z = D^{-1} y, the same recurrence as L^T x = D^{-1} y).
// TH threads per workgroup: one wavefront (64) for coarse meshes with
// ncx <= 32, where a pivot step has too little work to amortise a
// multi-wavefront barrier; 1024 above (three trailing entries per thread,
// four wavefronts per SIMD to overlap the latency of a pivot step, which is
// what bounds a batch of a few hundred samples with one workgroup per CU).
template <int NQ, bool PG, int TH>
__global__ __launch_bounds__(TH) void coarse_solve_kernel(CoarseArgs args) {
  constexpr int ES = PG ? 16 : 10;  // doubles per element matrix
  constexpr int BMX = TH == 64 ? COARSE_SMALL_B : COARSE_BMAX;
  static_assert(TH == 64 || TH == COARSE_THREADS, "workgroup sizes");
  constexpr int NE = (BMX * ES + TH - 1) / TH;  // element-row prefetch
  extern __shared__ double smem[];
  const int ncx = args.ncx, ncy = args.ncy;
  const int nix = ncx - 1, niy = ncy - 1, nU = nix * niy, B = ncx, WN = B + 1, FN = B + 2;
  double* Wn = smem;         // WN*WN: row r in slot r % WN, column c in slot c % WN
  double* F = Wn + WN * WN;  // FN: forward-substituted rhs, row r in slot r % FN
  double* Ec = F + FN;       // 3 x ncx x ES: ring of element rows of S (row e in slot e % 3)
  __shared__ int bad;
  __shared__ double colv[2][COARSE_BMAX];  // colv[j & 1][t - 1] = W(j + t, j), t = 1..B
  __shared__ double rowv[2][PG ? COARSE_BMAX : 1];  // PG: rowv[j & 1][t - 1] = W(j, j + t)
  __shared__ double pinv[2];               // pinv[j & 1] = 1 / d_j
  const int tid = threadIdx.x;
  const int Mc = ncx * ncy;
  const double H = 1.0 / ncx;
  // column j: [1/d_j, l_{j+1,j}, ..., l_{j+B,j}], then one zero
  double* Lc = args.work + (int64_t)blockIdx.x * ((int64_t)nU * WN + 1);
  const int64_t zero = (int64_t)nU * WN;
  if (tid == 0) Lc[zero] = 0.0;
  // entries (io >= ko) of the B x B trailing triangle handled by this lane,
  // the same for every pivot column, packed io | ko << 8 (io = B: unused)
  int tik[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = tid + TH * q;
    if (PG) {
      tik[q] = t < B * B ? ((t / B) | ((t % B) << 8)) : B;
    } else {
      int io = 0;
      while ((io + 1) * (io + 2) / 2 <= t) ++io;
      const bool used = t < B * (B + 1) / 2;
      tik[q] = used ? (io | ((t - io * (io + 1) / 2) << 8)) : B;
    }
  }

  // one sample per workgroup: its slice of the workspace must survive until
  // the backward kernel has read it
  {
    const int64_t s = blockIdx.x;
    if (s >= args.nsamples) return;
    const double* Ss = args.S + s * (int64_t)Mc * ES;
    double* Us = args.U + s * (int64_t)nU;
    for (int i = tid; i < WN * WN; i += blockDim.x) Wn[i] = 0.0;
    if (tid == 0) bad = 0;
    // Element rows of S go through an LDS ring of three.  Node row iy uses
    // element rows iy and iy + 1.  Rows 0..2 are loaded here; the first node
    // of node row iy >= 1 stores element row iy + 2 (prefetched into
    // registers a node row earlier) into the slot of row iy - 1, which only
    // node rows up to iy - 1 used, and prefetches element row iy + 3.
    double epre[NE];
    auto erow_fetch = [&](int e) {
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int t = tid + TH * k;
        epre[k] = (e < ncy && t < ncx * ES) ? Ss[(int64_t)e * ncx * ES + t] : 0.0;
      }
    };
    auto erow_store = [&](int e) {
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int t = tid + TH * k;
        if (e < ncy && t < ncx * ES) Ec[(e % 3) * ncx * ES + t] = epre[k];
      }
    };
    for (int e = 0; e < 3; ++e)
      if (e < ncy)
        for (int t = tid; t < ncx * ES; t += blockDim.x) Ec[e * ncx * ES + t] = Ss[(int64_t)e * ncx * ES + t];
    erow_fetch(3);

    // load of row r (the last thread keeps the next row's value)
    auto node_load = [&](int r) -> double {
      if (r >= nU) return 0.0;
      const int px = r % nix + 1, py = r / nix + 1;
      if (!args.load) return H * H;  // four elements, int_K p^l = H^2/4 each
      const double* L = args.load;
      return (L[((py - 1) * ncx + (px - 1)) * 4 + 2] + L[((py - 1) * ncx + px) * 4 + 3]) +
             (L[(py * ncx + (px - 1)) * 4 + 1] + L[(py * ncx + px) * 4 + 0]);
    };
    double bnext = tid == TH - 1 ? node_load(0) : 0.0;
    __syncthreads();

    // Row r of the coarse system: node (ix, iy) = grid node (px, py); its four
    // elements SW=(px-1,py-1), SE=(px,py-1), NW=(px-1,py), NE=(px,py) see it as
    // local node 2, 3, 1, 0 respectively.  The entry at offset B (the SW
    // coupling, column r - B) also goes to colB, the next pivot's column.
    // PG: the column above the diagonal, G[r - t][r], enters with the row
    // (and its entry at distance B goes to rowB, the next pivot's row).
    auto insert_row = [&](int r, double* colB, double* rowB) {
      const int ix = r % nix, iy = r / nix, px = ix + 1, py = iy + 1;
      if (ix == 0 && iy >= 1) {
        erow_store(iy + 2);
        erow_fetch(iy + 3);
      }
      const double* eS = Ec + ((py - 1) % 3) * ncx * ES;
      const double* eN = Ec + (py % 3) * ncx * ES;
      const double* sSW = eS + (px - 1) * ES;
      const double* sSE = eS + px * ES;
      const double* sNW = eN + (px - 1) * ES;
      const double* sNE = eN + px * ES;
      for (int t = tid; t <= B; t += TH) {
        // v = G[r][r - t] (test r, trial r - t), u = G[r - t][r]; local
        // indices of r and of the neighbour in each shared element
        double v = 0.0, u = 0.0;
        if (t == 0)
          v += (sget<PG>(sSW, 2, 2) + sget<PG>(sSE, 3, 3)) + (sget<PG>(sNW, 1, 1) + sget<PG>(sNE, 0, 0));
        if (t == 1 && ix >= 1) {
          v += sget<PG>(sSW, 3, 2) + sget<PG>(sNW, 0, 1);
          u += sget<PG>(sSW, 2, 3) + sget<PG>(sNW, 1, 0);
        }
        if (t == nix - 1 && iy >= 1 && ix <= nix - 2) {
          v += sget<PG>(sSE, 1, 3);
          u += sget<PG>(sSE, 3, 1);
        }
        if (t == nix && iy >= 1) {
          v += sget<PG>(sSW, 1, 2) + sget<PG>(sSE, 0, 3);
          u += sget<PG>(sSW, 2, 1) + sget<PG>(sSE, 3, 0);
        }
        if (t == nix + 1 && iy >= 1 && ix >= 1) {
          v += sget<PG>(sSW, 0, 2);
          u += sget<PG>(sSW, 2, 0);
        }
        if (r - t >= 0) {
          Wn[(r % WN) * WN + ((r - t) % WN)] = v;  // every entry of the row, once
          if (PG && t > 0) Wn[((r - t) % WN) * WN + (r % WN)] = u;
          if (t == B && colB) colB[B - 1] = v;
          if (PG && t == B && rowB) rowB[B - 1] = u;
        }
      }
      if (tid == TH - 1) {
        F[r % FN] = bnext;
        bnext = node_load(r + 1);
      }
    };

    const int r0 = B < nU - 1 ? B : nU - 1;
    for (int r = 0; r <= r0; ++r) {
      insert_row(r, nullptr, nullptr);
      __syncthreads();
    }
    // pivot 0's column and 1/d_0
    for (int t = 1 + tid; t <= r0; t += TH) {
      colv[0][t - 1] = Wn[t * WN];
      if (PG) rowv[0][t - 1] = Wn[t];
    }
    if (tid == 0) {
      const double d = Wn[0];
      pinv[0] = 1.0 / d;
      if (!(d > 0.0)) bad = 1;
    }
    __syncthreads();

    for (int j = 0; j < nU; ++j) {
      const int b = j & 1;
      const double inv = pinv[b];
      const int jj = j % WN;
      const int cnt = (j + B < nU - 1 ? j + B : nU - 1) - j;
      // rank-1 update of the trailing triangle, this lane's fixed entries:
      // all reads first, then all writes (distinct addresses), so that the
      // reads are not serialised behind possibly aliasing writes.  Entries
      // in the first column of the triangle are column j+1.
      {
        double wv[NQ];
        int idx[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int io = tik[q] & 255, ko = tik[q] >> 8;
          idx[q] = __umul24(wrap(jj + 1 + io, WN), WN) + wrap(jj + 1 + ko, WN);  // 24-bit: full rate
          wv[q] = (io < cnt && ko < cnt) ? Wn[idx[q]] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int io = tik[q] & 255, ko = tik[q] >> 8;
          if (io < cnt && ko < cnt) wv[q] -= colv[b][io] * inv * (PG ? rowv[b][ko] : colv[b][ko]);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int io = tik[q] & 255, ko = tik[q] >> 8;
          if (io < cnt && ko < cnt) {
            Wn[idx[q]] = wv[q];
            if (ko == 0) {
              if (io > 0) {
                colv[b ^ 1][io - 1] = wv[q];
              } else {
                pinv[b ^ 1] = 1.0 / wv[q];
                if (!(wv[q] > 0.0)) bad = 1;
              }
            } else if (PG && io == 0) {
              rowv[b ^ 1][ko - 1] = wv[q];
            }
          }
        }
      }
      // forward substitution step and column j of L (F[j] is final: every
      // pivot above it has been applied in an earlier phase)
      for (int t = 1 + tid; t <= cnt; t += TH) {
        const double l = colv[b][t - 1] * inv;
        Lc[(int64_t)j * WN + t] = PG ? rowv[b][t - 1] * inv : l;  // PG: (D^{-1} U)_{j, j+t}
        F[(j + t) % FN] -= l * F[j % FN];
      }
      if (tid == 0) {
        Lc[(int64_t)j * WN] = inv;
        Us[j] = F[j % FN] * inv;  // z_j = y_j / d_j, overwritten by x_j below
      }
      // the row entering the window takes the slot of row j (its last reader
      // was the phase before); its F slot is that of row j - 1
      if (j + 1 + B < nU) insert_row(j + 1 + B, colv[b ^ 1], PG ? rowv[b ^ 1] : nullptr);
      COARSE_SYNC();
    }
    if (tid == 0 && args.status) args.status[s] = bad ? STOMSFEM_ENOTSPD : STOMSFEM_OK;
  }
}

// Blocked forward pass for the symmetric system with 32 < B <= 64 (the
// pivot-per-barrier kernel above is bound by the latency of its per-pivot
// phase, not by arithmetic).  Panels of CB_NB pivots, 256 threads, one
// barrier per panel, software-pipelined one panel deep:
//   wavefront 0 applies the rank-CB_NB update of panel P-1 to the columns of
//      panel P, then factors panel P: every lane factors the CB_NB x CB_NB
//      diagonal block (broadcast LDS reads, no cross-lane traffic) and
//      eliminates its two rows j0 + lane and j0 + 64 + lane with it; l, the
//      unscaled entries of the rows below the panel, the block's l, 1/d and
//      z = D^{-1} y go to LDS (double-buffered), and it does the forward
//      substitution of the rhs.  It issues no global memory operation;
//   wavefronts 1-2 apply the update of panel P-1 to the rest of the
//      trailing triangle (columns past panel P), one 4 x 4 register tile per
//      lane, two 16-byte LDS reads per factor and pivot; wavefront 2 also
//      keeps the ring of element rows and the rhs of new rows;
//   wavefront 3 writes panel P-1's columns of L (one contiguous block) and z,
//      clears the slots of panel P-1's rows and writes into them the five
//      nonzero entries of each row first touched by panel P+1.
// Each entry receives the updates of its pivots in pivot order, each as
// w - (a_ip / d_p) a_kp.  The band window keeps row r in slot r mod
// (B + 2 NB) as [A_rr, A_r,r-1, ..., A_r,r-B]; element rows of S go through
// an LDS ring of three.  Accesses of masked-off lanes go to a junk slot
// instead of branching.  About 76 KB of LDS (gfx950 gives a workgroup up to
// 160 KB).
constexpr int CB_TH = 256;
constexpr int CB_NB = 8;
constexpr int CB_BMAX = 64;
constexpr int CB_NE = (CB_BMAX * 10 + 63) / 64;  // element-row prefetch per lane of wavefront 2

size_t coarse_blocked_lds_bytes(int ncx) {
  const int WN = ncx + 2 * CB_NB;
  return sizeof(double) * ((size_t)WN * (ncx + 1) + (size_t)WN + 3 * (size_t)ncx * 10);
}

__global__ __launch_bounds__(CB_TH) void coarse_blocked_kernel(CoarseArgs args) {
  constexpr int NB = CB_NB;
  extern __shared__ double smem[];
  const int ncx = args.ncx, ncy = args.ncy;
  const int nix = ncx - 1, nU = nix * (ncy - 1), B = ncx, WN = B + 2 * NB, BW = B + 1;
  double* Wb = smem;         // WN x BW: Wb[slot(r) BW + (r - c)] = A[r][c]
  double* F = Wb + WN * BW;  // WN: rhs, row r in slot(r)
  double* Ec = F + WN;       // 3 x ncx x 10: element row e in slot e % 3
  // per panel (buffer P & 1): Lp[pp][io] = l_{j0+NB+io, j0+pp} and Ap the
  // unscaled entry, Lq[pp][i] = l_{j0+i, j0+pp} (i > pp), 1/d_p, z_p
  __shared__ __align__(16) double Lp[2][NB][CB_BMAX];
  __shared__ __align__(16) double Ap[2][NB][CB_BMAX];
  __shared__ double Lq[2][NB][NB];
  __shared__ double dq[2][NB], zq[2][NB];
  __shared__ double Bk[NB][NB];  // the panel block after the previous panel's update (wavefront 0)
  __shared__ double junk[64];    // target of the masked-off lanes' accesses
  __shared__ double zero1;       // 0.0: the source of absent terms
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t s = blockIdx.x;
  if (s >= args.nsamples) return;
  const double* Ss = args.S + s * (int64_t)ncx * ncy * 10;
  double* Us = args.U + s * (int64_t)nU;
  double* Lc = args.work + s * ((int64_t)nU * BW + 1);  // column j: [1/d_j, l_{j+1,j}, ..., l_{j+B,j}]
  const double H = 1.0 / ncx;
  double* jk = &junk[lane];
  if (tid == 0) {
    Lc[(int64_t)nU * BW] = 0.0;
    bad = 0;
    zero1 = 0.0;
  }
  // x - WN while x >= WN, for 0 <= x < 3 WN
  auto wrapn = [&](int x) {
    x = x >= WN ? x - WN : x;
    return x >= WN ? x - WN : x;
  };
  // this lane's 4 x 4 tile (wavefronts 1-2) of the triangle of rows and
  // columns j0 + NB .. j0 + B - 1 (offsets 4 tr.., 4 tc.. from j0 + NB);
  // tmask bit 4a+b: entry (4tr+a, 4tc+b) lies in it
  const int TB = B - NB, nT = (TB + 3) / 4;
  int tr = 0;
  const int tix = lane + 64 * (wave - 1);
  while ((tr + 1) * (tr + 2) / 2 <= tix) ++tr;
  const int tc = tix - tr * (tr + 1) / 2;
  const bool tile = (wave == 1 || wave == 2) && tr < nT;
  unsigned tmask = 0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      if (4 * tr + a < TB && 4 * tc + b <= 4 * tr + a) tmask |= 1u << (4 * a + b);

  auto node_load = [&](int r) -> double {
    if (r >= nU) return 0.0;
    const int px = r % nix + 1, py = r / nix + 1;
    if (!args.load) return H * H;  // four elements, int_K p^l = H^2/4 each
    const double* L = args.load;
    return (L[((py - 1) * ncx + (px - 1)) * 4 + 2] + L[((py - 1) * ncx + px) * 4 + 3]) +
           (L[(py * ncx + (px - 1)) * 4 + 1] + L[(py * ncx + px) * 4 + 0]);
  };
  // nonzero entry e (0..4) of row r: offset t in {0, 1, nix-1, nix, nix+1}
  // (diagonal, W, SE, S, SW couplings) and its value, the sum of up to four
  // element-matrix entries around the node as in coarse_solve_kernel (absent
  // terms read an LDS zero, so every lane takes the same path)
  auto nonzero = [&](int r, int e, int& t, double& v) {
    const int ix = r % nix, iy = r / nix, px = ix + 1, py = iy + 1;
    const double* eS = Ec + ((py - 1) % 3) * ncx * 10;
    const double* eN = Ec + (py % 3) * ncx * 10;
    const double* sSW = eS + (px - 1) * 10;
    const double* sSE = eS + px * 10;
    const double* sNW = eN + (px - 1) * 10;
    const double* sNE = eN + px * 10;
    const double* z = &zero1;
    // packed indices: (0,0)=0 (0,1)=1 (0,2)=2 (0,3)=3 (1,1)=4 (1,2)=5 (1,3)=6 (2,2)=7 (2,3)=8 (3,3)=9
    const double *pa = z, *pb = z, *pc = z, *pd = z;
    t = e == 0 ? 0 : e == 1 ? 1 : e == 2 ? nix - 1 : e == 3 ? nix : nix + 1;
    if (e == 0) {
      pa = sSW + 7;  // (2,2)
      pb = sSE + 9;  // (3,3)
      pc = sNW + 4;  // (1,1)
      pd = sNE + 0;  // (0,0)
    }
    const bool c1 = e == 1 && ix >= 1, c3 = e == 3 && iy >= 1;
    pa = c1 ? sSW + 8 : c3 ? sSW + 5 : pa;  // (3,2) / (1,2)
    pb = c1 ? sNW + 1 : c3 ? sSE + 3 : pb;  // (0,1) / (0,3)
    pa = (e == 2 && iy >= 1 && ix <= nix - 2) ? sSE + 6 : pa;  // (1,3)
    pa = (e == 4 && iy >= 1 && ix >= 1) ? sSW + 2 : pa;        // (0,2)
    v = (*pa + *pb) + (*pc + *pd);
  };
  double epre[CB_NE];
  auto erow_fetch = [&](int e) {  // wavefront 2
#pragma unroll
    for (int k = 0; k < CB_NE; ++k) {
      const int t = lane + 64 * k;
      epre[k] = (e < ncy && t < ncx * 10) ? Ss[(int64_t)e * ncx * 10 + t] : 0.0;
    }
  };
  auto erow_store = [&](int e) {
#pragma unroll
    for (int k = 0; k < CB_NE; ++k) {
      const int t = lane + 64 * k;
      if (e < ncy && t < ncx * 10) Ec[(e % 3) * ncx * 10 + t] = epre[k];
    }
  };

  // prologue: element rows 0..2, the cleared window, rows 0 .. NB+B-1 and
  // their rhs
  for (int e = 0; e < 3 && e < ncy; ++e)
    for (int t = tid; t < ncx * 10; t += CB_TH) Ec[e * ncx * 10 + t] = Ss[(int64_t)e * ncx * 10 + t];
  for (int i = tid; i < WN * BW; i += CB_TH) Wb[i] = 0.0;
  int eld = ncy - 1 < 2 ? ncy - 1 : 2;  // highest element row in the ring
  if (wave == 2) erow_fetch(eld + 1);
  __syncthreads();
  for (int i = tid; i < (NB + B) * 5; i += CB_TH) {
    const int r = i / 5, e = i - 5 * r;
    int t;
    double v;
    if (r < nU) {
      nonzero(r, e, t, v);
      if (r - t >= 0) Wb[r * BW + t] = v;
    }
  }
  for (int r = tid; r < NB + B; r += CB_TH)
    if (r < nU) F[r] = node_load(r);
  double fnext = (wave == 2 && lane < NB) ? node_load(NB + B + lane) : 0.0;
  __syncthreads();

  int sj = 0;  // slot of row j0
  for (int P = 0;; ++P) {
    const int j0 = P * NB;
    if (j0 - NB >= nU) break;
    const int cb = P & 1, pb = cb ^ 1;  // buffers of panels P and P-1
    if (wave == 0 && j0 < nU) {
      // rows R1 = j0 + lane and R2 = j0 + 64 + lane; entry (R, j0 + k) in x[k]
      const bool h1 = lane < NB + B && j0 + lane < nU;
      const bool h2 = 64 + lane < NB + B && j0 + 64 + lane < nU;
      const int s1 = wrapn(sj + lane), s2 = wrapn(sj + (64 + lane < NB + B ? 64 + lane : 0));
      double x1[NB], x2[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const bool v1 = h1 && lane >= k && lane - k <= B, v2 = h2 && 64 + lane - k <= B;
        const double y1 = *(v1 ? &Wb[s1 * BW + (lane - k)] : jk);
        const double y2 = *(v2 ? &Wb[s2 * BW + (64 + lane - k)] : jk);
        x1[k] = v1 ? y1 : 0.0;
        x2[k] = v2 ? y2 : 0.0;
      }
      const double g1 = *(h1 ? &F[s1] : jk), g2 = *(h2 ? &F[s2] : jk);
      double f1 = h1 ? g1 : 0.0, f2 = h2 ? g2 : 0.0;
      if (P >= 1) {
        // the update of panel P-1 on these columns: row j0 + lane is its
        // row offset io = lane (rows j0 + 64 + lane are past its reach)
        const bool in = lane < B;
#pragma unroll
        for (int pp = 0; pp < NB; ++pp) {
          const double lv = *(in ? &Lp[pb][pp][lane] : jk);
          const double l = in ? lv : 0.0;
#pragma unroll
          for (int k = 0; k < NB; ++k) x1[k] -= l * Ap[pb][pp][k];
        }
      }
      // the diagonal block (rows and columns j0 .. j0 + NB - 1) and the rhs
      // of its rows in every lane: lanes 0 .. NB-1 hold the block rows, the
      // other lanes read them back (same addresses: broadcast); rows past nU
      // are an identity block so that no pivot is zero there
#pragma unroll
      for (int k = 0; k < NB; ++k) *(lane < NB && k <= lane ? &Bk[lane][k] : jk) = x1[k];
      double blk[NB][NB], fb[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const bool in = j0 + i < nU;
#pragma unroll
        for (int k = 0; k <= i; ++k) blk[i][k] = in ? Bk[i][k] : (i == k ? 1.0 : 0.0);
        const double v = *(in ? &F[wrapn(sj + i)] : jk);
        fb[i] = in ? v : 0.0;
      }
      // every lane factors the block (right-looking, pivot order) and
      // carries its own two rows along: entry (R, j0 + k) receives the
      // update of pivot p as x - (x_p / d_p) A_{j0+k, p}, in pivot order
      double dinv[NB], yv[NB], l1s[NB], l2s[NB];
#pragma unroll
      for (int pp = 0; pp < NB; ++pp) {
        const double d = blk[pp][pp];
        // 1/d: hardware reciprocal and two Newton steps (within an ulp or
        // two; the pivot chain runs through it)
        double inv = __builtin_amdgcn_rcp(d);
        inv = fma(fma(-d, inv, 1.0), inv, inv);
        inv = fma(fma(-d, inv, 1.0), inv, inv);
        dinv[pp] = inv;
        if (j0 + pp < nU && !(d > 0.0)) bad = 1;
        const double y = fb[pp];
        yv[pp] = y;
#pragma unroll
        for (int i = pp + 1; i < NB; ++i) {
          const double li = blk[i][pp] * inv;
          fb[i] -= li * y;
#pragma unroll
          for (int k = pp + 1; k <= i; ++k) blk[i][k] -= li * blk[k][pp];
        }
        const bool b1 = h1 && lane > pp && lane - pp <= B, b2 = h2 && 64 + lane - pp <= B;
        const double l1 = b1 ? x1[pp] * inv : 0.0, l2 = b2 ? x2[pp] * inv : 0.0;
        f1 -= l1 * y;
        f2 -= l2 * y;
#pragma unroll
        for (int k = pp + 1; k < NB; ++k) {
          x1[k] -= l1 * blk[k][pp];
          x2[k] -= l2 * blk[k][pp];
        }
        l1s[pp] = l1;
        l2s[pp] = l2;
      }
      // for the next step: the panel columns of the rows below the panel
      // (their factor is zero where the entry is outside the band, and so is
      // the entry), the block's factors, 1/d and z
#pragma unroll
      for (int pp = 0; pp < NB; ++pp) {
        *(lane >= NB ? &Lp[cb][pp][lane - NB] : jk) = l1s[pp];
        *(lane >= NB ? &Ap[cb][pp][lane - NB] : jk) = l1s[pp] != 0.0 ? x1[pp] : 0.0;
        if (64 + lane - NB < B) {
          Lp[cb][pp][64 + lane - NB] = l2s[pp];
          Ap[cb][pp][64 + lane - NB] = l2s[pp] != 0.0 ? x2[pp] : 0.0;
        }
        *(lane < NB && lane > pp ? &Lq[cb][pp][lane] : jk) = l1s[pp];
      }
      if (lane < NB) {
        double di = dinv[0], z = yv[0] * dinv[0];
#pragma unroll
        for (int pp = 1; pp < NB; ++pp) {
          di = lane == pp ? dinv[pp] : di;
          z = lane == pp ? yv[pp] * dinv[pp] : z;
        }
        dq[cb][lane] = di;
        zq[cb][lane] = z;  // z_p = y_p / d_p, overwritten by x_p in the backward pass
      }
      if (h1 && lane >= NB) F[s1] = f1;
      if (h2) F[s2] = f2;
    }
    if (tile && P >= 1) {
      // update of panel P-1 on rows / columns j0 + NB + 4 tr.. / 4 tc..:
      // offsets NB + 4 tr.. in its buffers
      double w[4][4];
      double* pa[4][4];
      unsigned vm = tmask;  // entries inside the triangle and the system
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (j0 + NB + 4 * tr + a >= nU) vm &= ~(15u << (4 * a));
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int sa = wrapn(sj + NB + 4 * tr + a) * BW + 4 * (tr - tc) + a;  // slot(i) BW + (i - k) for b = 0
#pragma unroll
        for (int b = 0; b < 4; ++b) pa[a][b] = (vm >> (4 * a + b) & 1u) ? &Wb[sa - b] : jk;
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) w[a][b] = *pa[a][b];
#pragma unroll
      for (int pp = 0; pp < NB; ++pp) {
        const double2 la = *reinterpret_cast<const double2*>(&Lp[pb][pp][NB + 4 * tr]);
        const double2 lb = *reinterpret_cast<const double2*>(&Lp[pb][pp][NB + 4 * tr + 2]);
        const double2 aa = *reinterpret_cast<const double2*>(&Ap[pb][pp][NB + 4 * tc]);
        const double2 ab = *reinterpret_cast<const double2*>(&Ap[pb][pp][NB + 4 * tc + 2]);
        const double l[4] = {la.x, la.y, lb.x, lb.y}, av[4] = {aa.x, aa.y, ab.x, ab.y};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) w[a][b] -= l[a] * av[b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) *pa[a][b] = w[a][b];
    }
    const int rb = j0 + NB + B;  // rows first touched by panel P+1
    const int so = wrapn(sj + WN - NB);  // slot of row j0 - NB: panel P-1's rows
    if (wave == 2) {
      // rhs of the new rows (prefetched a step ahead); element ring: the
      // rows assembled in the next step need element rows up to
      // iy(last) + 1, and the slot written here holds a row no longer read
      if (lane < NB && rb + lane < nU) F[wrapn(so + lane)] = fnext;
      fnext = lane < NB ? node_load(rb + lane + NB) : 0.0;
      const int rl = j0 + 3 * NB + B - 1 < nU - 1 ? j0 + 3 * NB + B - 1 : nU - 1;
      if (rl / nix + 1 > eld && eld + 1 < ncy) {
        erow_store(eld + 1);
        ++eld;
        erow_fetch(eld + 1);
      }
    } else if (wave == 3) {
      if (P >= 1) {
        // columns j0 - NB .. j0 - 1 of L (a contiguous block of the
        // workspace) and their z
        const int jp = j0 - NB, ncol = nU - jp < NB ? nU - jp : NB;
        double* Lb = Lc + (int64_t)jp * BW;
#pragma unroll
        for (int pp = 0; pp < NB; ++pp) {
          if (pp < ncol) {
            for (int t = lane; t < BW; t += 64) {
              const double* src =
                  t == 0 ? &dq[pb][pp] : (t < NB - pp ? &Lq[pb][pp][pp + t] : &Lp[pb][pp][t - (NB - pp)]);
              Lb[pp * BW + t] = *src;
            }
          }
        }
        if (lane < ncol) Us[jp + lane] = zq[pb][lane];
      }
      // panel P-1's row slots: cleared, then the nonzeros of the rows first
      // touched by panel P+1 (LDS operations of one wavefront complete in
      // order)
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        double* row = Wb + wrapn(so + q) * BW;
        for (int t = lane; t < BW; t += 64) row[t] = 0.0;
      }
      if (lane < 5 * NB) {
        const int q = lane / 5, r = rb + q;
        int t = 0;
        double v = 0.0;
        if (r < nU) nonzero(r, lane - 5 * q, t, v);
        *(r < nU && r - t >= 0 ? &Wb[wrapn(so + q) * BW + t] : jk) = v;
      }
    }
    sj = wrapn(sj + NB);
    COARSE_SYNC();
  }
  if (tid == 0 && args.status) args.status[s] = bad ? STOMSFEM_ENOTSPD : STOMSFEM_OK;
}

// Backward substitution L^T x = z for the samples of one forward launch: one
// wavefront per sample (workgroup slice blockIdx.x of the workspace).
template <bool FAR>
__global__ __launch_bounds__(64) void coarse_back_kernel(CoarseArgs args) {
  const int ncx = args.ncx, ncy = args.ncy;
  const int nU = (ncx - 1) * (ncy - 1), B = ncx, WN = B + 1;
  const int64_t s = blockIdx.x;
  if (s >= args.nsamples) return;
  const double* Lc = args.work + s * ((int64_t)nU * WN + 1);
  const int64_t zero = (int64_t)nU * WN;
  double* Us = args.U + s * (int64_t)nU;
  const int lam = threadIdx.x;
  const int kt = (nU - 1) >> 6;
  auto yload = [&](int k) -> double {
    const int i = 64 * k + lam;
    return (k >= 0 && i < nU) ? Us[i] : 0.0;
  };
  // yc, y1, y2: blocks k, k-1, k-2 (y2 only if FAR); yp: the next block to
  // enter, loaded one block ahead
  double yc = yload(kt), y1 = yload(kt - 1), y2 = FAR ? yload(kt - 2) : 0.0;
  double yp = yload(FAR ? kt - 3 : kt - 2);
  BackStep pf[COARSE_PD];
#pragma unroll
  for (int d = 0; d < COARSE_PD; ++d) pf[d] = back_loads<FAR>(Lc, zero, WN, B, nU, 64 * kt + 63 - d, lam);
  for (int k = kt; k >= 0; --k) {
    double xs = 0.0;
    // groups of COARSE_PD steps; step j issues the loads of step
    // j - COARSE_PD, and the empty asm statements keep the compiler from
    // moving them next to their use
#pragma unroll 1
    for (int u0 = 63; u0 >= 0; u0 -= COARSE_PD) {
#pragma unroll
      for (int d = 0; d < COARSE_PD; ++d) {
        const int u = u0 - d, j = 64 * k + u;
        if (j < nU) {
          const double x = lane_value(yc, u);
          xs = lam == u ? x : xs;
          yc = __builtin_fma(-pf[d].lc, x, yc);
          y1 = __builtin_fma(-pf[d].l1, x, y1);
          if (FAR) y2 = __builtin_fma(-pf[d].l2, x, y2);
        }
        // the slot is free again: load step j - COARSE_PD into it
        pf[d] = back_loads<FAR>(Lc, zero, WN, B, nU, j - COARSE_PD, lam);
        __asm__ volatile("" ::: "memory");
      }
    }
    if (64 * k + lam < nU) Us[64 * k + lam] = xs;
    yc = y1;
    if (FAR) {
      y1 = y2;
      y2 = yp;
      yp = yload(k - 4);
    } else {
      y1 = yp;
      yp = yload(k - 3);
    }
  }
}

// qoi_mean[i] = (1/N) sum_s U[s][i]; qoi_var[i] = (1/N) sum_s U^2 - mean^2.
// Two passes with a fixed summation order (bitwise reproducible): partial
// sums over chunks of CS samples (64 unknowns per workgroup, the four
// wavefronts taking every fourth sample of the chunk, combined in order),
// then the chunks in order.  Reads are coalesced along the unknowns.
constexpr int QOI_TY = 4;

__global__ __launch_bounds__(64 * QOI_TY) void qoi_partial_kernel(int64_t N, int nU, int64_t CS, const double* U,
                                                                  double* part) {
  __shared__ double sh[2][QOI_TY][64];
  const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + x;
  const int64_t c = blockIdx.y, s0 = c * CS, s1 = s0 + CS < N ? s0 + CS : N;
  double m1 = 0.0, m2 = 0.0;
  if (i < nU)
    for (int64_t s = s0 + y; s < s1; s += QOI_TY) {
      const double u = U[s * nU + i];
      m1 += u;
      m2 += u * u;
    }
  sh[0][y][x] = m1;
  sh[1][y][x] = m2;
  __syncthreads();
  if (y == 0 && i < nU) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int k = 0; k < QOI_TY; ++k) {
      a += sh[0][k][x];
      b += sh[1][k][x];
    }
    part[(c * nU + i) * 2] = a;
    part[(c * nU + i) * 2 + 1] = b;
  }
}

__global__ void qoi_final_kernel(int64_t N, int nU, int64_t nch, const double* part, double* mean, double* var) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nU) return;
  double m1 = 0.0, m2 = 0.0;
  for (int64_t c = 0; c < nch; ++c) {
    m1 += part[(c * nU + i) * 2];
    m2 += part[(c * nU + i) * 2 + 1];
  }
  const double inv = N > 0 ? 1.0 / (double)N : 0.0;
  m1 *= inv;
  m2 *= inv;
  if (mean) mean[i] = m1;
  if (var) var[i] = m2 - m1 * m1;
}

// samples per QoI chunk: at most 1024 chunks
static int64_t qoi_chunk(int64_t N) {
  const int64_t cs = (N + 1023) / 1024;
  return cs < 64 ? 64 : cs;
}

static bool use_blocked(int ncx, bool pg) { return !pg && ncx > COARSE_SMALL_B && ncx <= CB_BMAX; }

size_t coarse_lds_bytes(int ncx, bool pg) {
  if (use_blocked(ncx, pg)) return coarse_blocked_lds_bytes(ncx);
  const int WN = ncx + 1;
  return sizeof(double) * ((size_t)WN * WN + (size_t)WN + 1 + 3 * (size_t)ncx * (pg ? 16 : 10));
}

int64_t coarse_grid(int64_t nsamples) { return nsamples < 4096 ? nsamples : 4096; }

// Samples per launch: 4096 workgroups for the workgroup-per-sample kernels;
// the one-lane-per-sample kernel of small square meshes takes up to 65536
// (1024 wavefronts; its workspace is about 3.5 KB per sample).
static int64_t coarse_chunk(int ncx, int ncy, int64_t nsamples) {
  const int64_t cap = (ncx == ncy && ncx <= 8) ? 65536 : 4096;
  return nsamples < cap ? nsamples : cap;
}

int64_t coarse_work_doubles(int ncx, int ncy, int64_t nsamples) {
  return coarse_chunk(ncx, ncy, nsamples) * ((int64_t)(ncx - 1) * (ncy - 1) * (ncx + 1) + 1);
}

// Small square coarse meshes (ncx = ncy = NC <= 8, the symmetric system):
// one lane per sample.  With NU = (NC-1)^2 unknowns and half-bandwidth
// B = NC (couplings at offsets 1, NC-2, NC-1, NC), every row, window slot
// and band offset is a compile-time constant, so the factor window lives in
// registers.  Row r is assembled from the four elements around its node as
// in coarse_solve_kernel, then eliminated by Crout's LDL^T,
//   u_rc = A_rc - sum_{j<c} u_rj l_cj,  l_rc = u_rc / d_c,  d_r = A_rr - sum_c l_rc u_rc,
// with the forward substitution y_r = b_r - sum_c l_rc y_c alongside.  The
// band of L and z = D^{-1} y go to the workspace at [(r B + k) n + s] and
// [(NU B + r) n + s] (coalesced across the lanes), and the backward pass
// x_r = z_r - sum_{i=r+1}^{r+B} l_ir x_i reads them back.  Status ENOTSPD if
// a pivot is not positive (or NaN).
template <int NC>
__global__ __launch_bounds__(64) void coarse_lane_kernel(CoarseArgs a) {
  constexpr int n = NC - 1, NU = n * n, B = NC;
  const int64_t s = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (s >= a.nsamples) return;
  const int64_t ns = a.nsamples;
  const double* Ss = a.S + s * (int64_t)(NC * NC * 10);
  // workspace cursors: the band of L in store order (r B + k), then z
  double* wl = a.work + s;
  double* wz = a.work + (int64_t)NU * B * ns + s;
  const double H = 1.0 / NC;
  double Lw[B + 1][B];  // Lw[c % (B+1)][k] = l_{c, c-1-k}
  double Di[B + 1];     // 1 / d_c
  double Yw[B + 1];     // y_c
  bool bad = false;
#pragma clang loop unroll(full)
  for (int r = 0; r < NU; ++r) {
    // keeps each row's element-matrix loads next to their use (hoisting all
    // of them ahead of the elimination would exhaust the registers)
    asm volatile("" ::: "memory");
    const int ix = r % n, iy = r / n, px = ix + 1, py = iy + 1;
    const double* sSW = Ss + ((py - 1) * NC + (px - 1)) * 10;
    const double* sSE = Ss + ((py - 1) * NC + px) * 10;
    const double* sNW = Ss + (py * NC + (px - 1)) * 10;
    const double* sNE = Ss + (py * NC + px) * 10;
    double ar[B + 1];  // ar[t] = A[r][r - t]
#pragma unroll
    for (int t = 0; t <= B; ++t) ar[t] = 0.0;
    ar[0] = (selem(sSW, 2, 2) + selem(sSE, 3, 3)) + (selem(sNW, 1, 1) + selem(sNE, 0, 0));
    if (ix >= 1) ar[1] += selem(sSW, 3, 2) + selem(sNW, 0, 1);
    if (iy >= 1 && ix <= n - 2) ar[n - 1] += selem(sSE, 1, 3);
    if (iy >= 1) ar[n] += selem(sSW, 1, 2) + selem(sSE, 0, 3);
    if (iy >= 1 && ix >= 1) ar[n + 1] += selem(sSW, 0, 2);
    double b = H * H;
    if (a.load) {
      const double* L = a.load;
      b = (L[((py - 1) * NC + (px - 1)) * 4 + 2] + L[((py - 1) * NC + px) * 4 + 3]) +
          (L[(py * NC + (px - 1)) * 4 + 1] + L[(py * NC + px) * 4 + 0]);
    }
    double lr[B], ur[B];  // k: column c = r - 1 - k
#pragma unroll
    for (int k = B - 1; k >= 0; --k) {
      const int c = r - 1 - k;
      if (c < 0) {
        lr[k] = ur[k] = 0.0;
        continue;
      }
      double v = ar[k + 1];
#pragma unroll
      for (int k2 = B - 1; k2 > k; --k2) {
        if (r - 1 - k2 < 0) continue;
        v -= ur[k2] * Lw[c % (B + 1)][k2 - k - 1];  // l_{c, j}, j = r - 1 - k2
      }
      ur[k] = v;
      lr[k] = v * Di[c % (B + 1)];
    }
    double d = ar[0], y = b;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      if (r - 1 - k < 0) continue;
      d -= lr[k] * ur[k];
      y -= lr[k] * Yw[(r - 1 - k) % (B + 1)];
    }
    bad = bad || !(d > 0.0);
    const double di = 1.0 / d;
    Di[r % (B + 1)] = di;
    Yw[r % (B + 1)] = y;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      Lw[r % (B + 1)][k] = lr[k];
      *wl = lr[k];
      wl += ns;
    }
    *wz = y * di;
    wz += ns;
  }
  double X[B + 1];  // x_i, slot i % (B+1)
#pragma clang loop unroll(full)
  for (int r = NU - 1; r >= 0; --r) {
    asm volatile("" ::: "memory");
    wz -= ns;
    double x = *wz;
    // l_{i r} for i = r+1 .. r+B sits at index i B + (i - 1 - r): stride B + 1
    const double* li = a.work + ((int64_t)r * B + B) * ns + s;
#pragma unroll
    for (int i = r + 1; i <= r + B; ++i) {
      if (i < NU) x -= *li * X[i % (B + 1)];
      li += (B + 1) * ns;
    }
    X[r % (B + 1)] = x;
    a.U[s * NU + r] = x;
  }
  if (a.status) a.status[s] = bad ? STOMSFEM_ENOTSPD : STOMSFEM_OK;
}

template <int NC>
static void launch_lane(const CoarseArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(coarse_lane_kernel<NC>, dim3((unsigned)((a.nsamples + 63) / 64)), dim3(64), 0, st, a);
}

// work_cap = 0: the workspace holds coarse_work_doubles(ncx, ncy, N); else
// it holds work_cap doubles, and the chunks of samples and of the QoI
// partial sums are cut to fit (the caller has checked that one sample does).
static hipError_t launch_coarse_any(int ncx, int ncy, int64_t N, const double* S, const double* load, double* U,
                                    double* mean, double* var, int32_t* status, double* work, hipStream_t st,
                                    bool pg, int64_t work_cap = 0) {
  const int nU = (ncx - 1) * (ncy - 1);
  if (pg ? ncx > COARSE_PG_BMAX : (ncx * (ncx + 1) / 2 > COARSE_THREADS * COARSE_NQ || ncx > COARSE_BMAX))
    return hipErrorInvalidValue;
  const int ES = pg ? 16 : 10;
  if (N > 0 && nU > 0) {
    const bool small = ncx <= COARSE_SMALL_B;
    const int TH = small ? 64 : COARSE_THREADS;
    const int need = pg ? (ncx * ncx + TH - 1) / TH : (ncx * (ncx + 1) / 2 + TH - 1) / TH;
    const size_t lds = coarse_lds_bytes(ncx, pg);
    // samples per launch (pair): the workspace holds their factors
    int64_t chunk = (!pg && ncx == ncy && ncx <= 8) ? coarse_chunk(ncx, ncy, N) : coarse_grid(N);
    if (work_cap > 0) {
      const int64_t per = (int64_t)nU * (ncx + 1) + 1;
      if (per > work_cap) return hipErrorInvalidValue;
      if (chunk > work_cap / per) chunk = work_cap / per;
    }
    for (int64_t c = 0; c < N; c += chunk) {
      const int64_t n = N - c < chunk ? N - c : chunk;
      CoarseArgs a{ncx, ncy, n, S + c * (int64_t)ncx * ncy * ES, load, U + c * (int64_t)nU,
                   status ? status + c : nullptr, work};
      if (!pg && ncx == ncy && ncx <= 8) {
        // one lane per sample (the workspace holds n (nU (ncx+1) + 1) doubles)
        switch (ncx) {
          case 2: launch_lane<2>(a, st); break;
          case 3: launch_lane<3>(a, st); break;
          case 4: launch_lane<4>(a, st); break;
          case 5: launch_lane<5>(a, st); break;
          case 6: launch_lane<6>(a, st); break;
          case 7: launch_lane<7>(a, st); break;
          default: launch_lane<8>(a, st); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        continue;
      }
      const dim3 grid((unsigned)n), block(TH);
      if (small) {
        if (pg) {
          if (need <= 4)
            hipLaunchKernelGGL((coarse_solve_kernel<4, true, 64>), grid, block, lds, st, a);
          else
            hipLaunchKernelGGL((coarse_solve_kernel<16, true, 64>), grid, block, lds, st, a);
        } else {
          if (need <= 2)
            hipLaunchKernelGGL((coarse_solve_kernel<2, false, 64>), grid, block, lds, st, a);
          else
            hipLaunchKernelGGL((coarse_solve_kernel<9, false, 64>), grid, block, lds, st, a);
        }
      } else if (pg) {
        hipLaunchKernelGGL((coarse_solve_kernel<4, true, COARSE_THREADS>), grid, block, lds, st, a);
      } else if (use_blocked(ncx, pg)) {
        // the kernel's dynamic-LDS limit raised before each launch (a host call;
        // it then holds on whichever device is current)
        const hipError_t attr = hipFuncSetAttribute((const void*)coarse_blocked_kernel,
                                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                                    (int)coarse_blocked_lds_bytes(CB_BMAX));
        if (attr != hipSuccess) return attr;
        hipLaunchKernelGGL(coarse_blocked_kernel, grid, dim3(CB_TH), lds, st, a);
      } else {
        hipLaunchKernelGGL((coarse_solve_kernel<COARSE_NQ, false, COARSE_THREADS>), grid, block, lds, st, a);
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      if (ncx > 64)
        hipLaunchKernelGGL(coarse_back_kernel<true>, grid, dim3(64), 0, st, a);
      else
        hipLaunchKernelGGL(coarse_back_kernel<false>, grid, dim3(64), 0, st, a);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if ((mean || var) && nU > 0) {
    // the partial sums reuse the workspace of the factors (idle once the
    // backward passes, queued before on the same stream, are done):
    // 2 nch nU <= 3 min(N, 4096) nU doubles
    int64_t CS = qoi_chunk(N);
    if (work_cap > 0 && N > 0) {  // 2 nch nU partial sums must fit
      const int64_t nch_max = work_cap / (2 * (int64_t)nU);
      if (nch_max < 1) return hipErrorInvalidValue;
      if ((N + CS - 1) / CS > nch_max) CS = (N + nch_max - 1) / nch_max;
    }
    const int64_t nch = N > 0 ? (N + CS - 1) / CS : 0;
    if (nch > 0) {
      hipLaunchKernelGGL(qoi_partial_kernel, dim3((unsigned)((nU + 63) / 64), (unsigned)nch), dim3(64 * QOI_TY), 0,
                         st, N, nU, CS, U, work);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(qoi_final_kernel, dim3((nU + 255) / 256), dim3(256), 0, st, N, nU, nch, work, mean, var);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_coarse(int ncx, int ncy, int64_t N, const double* S, const double* load, double* U,
                         double* mean, double* var, int32_t* status, double* work, hipStream_t st) {
  return launch_coarse_any(ncx, ncy, N, S, load, U, mean, var, status, work, st, false);
}

// The same solve in a fixed workspace of work_cap doubles (samples and QoI
// partial sums in chunks that fit).
hipError_t launch_coarse_capped(int ncx, int ncy, int64_t N, const double* S, const double* load, double* U,
                                double* mean, double* var, int32_t* status, double* work, int64_t work_cap,
                                hipStream_t st) {
  if (work_cap < 1) return hipErrorInvalidValue;
  return launch_coarse_any(ncx, ncy, N, S, load, U, mean, var, status, work, st, false, work_cap);
}

// Petrov-Galerkin coarse system: S16 [N][ncx*ncy][16], S[trial][test] per element.
hipError_t launch_coarse_pg(int ncx, int ncy, int64_t N, const double* S16, const double* load, double* U,
                            double* mean, double* var, int32_t* status, double* work, hipStream_t st) {
  return launch_coarse_any(ncx, ncy, N, S16, load, U, mean, var, status, work, st, true);
}

// Element loads b^K_l = int_K b p^l of a bilinear source
// b = f00 + f10 x + f01 y + f11 x y (Sec. 5.3 takes 2 + x1 x2), for square
// elements of side H = 1/ncx, local nodes counter-clockwise from the
// lower-left corner.  b p^l is at most quadratic in each variable, so the
// 2 x 2 Gauss rule on K is exact.  One thread per element.
__global__ void element_loads_kernel(int ncx, int ncy, double f00, double f10, double f01, double f11,
                                     double* __restrict__ load) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncx * ncy) return;
  const double H = 1.0 / ncx;
  const double x0 = (e % ncx) * H, y0 = (e / ncx) * H;
  const double g[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  double b[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const double s = g[i], t = g[j], x = x0 + H * s, y = y0 + H * t;
      const double w = 0.25 * H * H * (f00 + f10 * x + f01 * y + f11 * x * y);
      b[0] += w * (1.0 - s) * (1.0 - t);
      b[1] += w * s * (1.0 - t);
      b[2] += w * s * t;
      b[3] += w * (1.0 - s) * t;
    }
  for (int l = 0; l < 4; ++l) load[4 * e + l] = b[l];
}

hipError_t launch_element_loads(int ncx, int ncy, const double* f, double* load, hipStream_t st) {
  const int n = ncx * ncy;
  hipLaunchKernelGGL(element_loads_kernel, dim3((n + 255) / 256), dim3(256), 0, st, ncx, ncy, f[0], f[1], f[2], f[3],
                     load);
  return hipGetLastError();
}

}  // namespace stomsfem
