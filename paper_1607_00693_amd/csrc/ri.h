// Random interpolation of the upscaled stiffness (Sec. 3.1, Algorithms 1
// and 2): kernel arguments and launchers.
#pragma once
#include "common.h"

namespace stomsfem {

constexpr int RI_KMAX = 4;   // local variables per patch
constexpr int RI_NN_MIN = 2;  // nodes per variable
constexpr int RI_NN_MAX = 9;

// Node set of one RI model: patch K owns the table rows off[K] .. off[K+1]-1,
// nn^nlv[K] of them; row c holds S_K at the tensor node whose digit for local
// variable i is (c / nn^(k-1-i)) mod nn (variable 0 slowest), node value
// t_d = lo + (cos(pi d / (nn-1)) + 1) (hi - lo) / 2.
struct RiNodeArgs {
  int32_t npatch, nxi, nn;
  double lo, hi;
  const int64_t* off;   // [npatch + 1]
  const int32_t* lv;    // [npatch][RI_KMAX]
  const int32_t* nlv;   // [npatch]
  int64_t start, count;  // table rows start .. start+count-1
  double* xi_out;       // [count][nxi]
  int64_t* pairs_out;   // [count]: i * npatch + K
};

// Coefficient blocks of listed (sample, patch) pairs p = s * npatch + K,
// regenerated from xi: out[i][m][m] (row-major, y outer).
struct RegenArgs {
  int32_t ncx, ncy, m, nxi;
  BumpParams bp;
  // channels-and-inclusions medium instead of the bump family when fmap is
  // set: fmap [ncy*m][ncx*m] feature per fine element (-1: background 1),
  // conductivity feature_theta(xi_j, decades)
  const int32_t* fmap;
  double decades;
  const int64_t* pairs;  // [count]
  int64_t count;
  const double* xi;      // [..][nxi]
  double* out;
};

// Online evaluation.  Pairs with a local variable outside [lo, hi] (or NaN)
// are appended to list (count via *list_count) for the plain solve.
struct RiApplyArgs {
  int32_t npatch, nxi, nn;
  int32_t ne;           // entries per table row and per S: 10 (symmetric) or 16 (Petrov-Galerkin); 0 = 10
  int64_t nsamples;
  double lo, hi;
  const double* table;  // [rows][ne]
  const int64_t* off;
  const int32_t* lv;
  const int32_t* nlv;
  const double* xi;     // [nsamples][nxi]
  double* S;            // [nsamples][npatch][ne]
  int32_t* status;      // [nsamples][npatch] or nullptr
  int64_t* list;
  unsigned long long* list_count;
};

hipError_t launch_ri_nodes(const RiNodeArgs& a, hipStream_t st);
hipError_t launch_regen_blocks(const RegenArgs& a, hipStream_t st);
hipError_t launch_ri_apply(const RiApplyArgs& a, hipStream_t st);
// S[pairs[i]] = Sc[i] (ne entries each), status[pairs[i]] = (stc[i] != 0 ? stc[i] : code).
hipError_t launch_scatter_pairs(const int64_t* pairs, int64_t count, const double* Sc, const int32_t* stc,
                                double* S, int32_t* status, int32_t code, hipStream_t st, int ne = 10);
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t st);

}  // namespace stomsfem
