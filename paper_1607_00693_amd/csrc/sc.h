// Sparse-grid stochastic collocation with search-and-plug-in dictionaries
// (Sec. 4.1.2, global SC methods): host construction of the Smolyak
// Clenshaw-Curtis grid, and the device kernels of the online stage.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <vector>

namespace stomsfem {

constexpr int SC_LEVEL_MAX = 8;  // digits up to 2^8

// Intervals of the finest one-dimensional grid of a level: 2^max(level, 1).
inline int sc_digit_base(int level) { return 1 << (level < 1 ? 1 : level); }

// Number of multi-indices of the combination formula (a size guard):
// binom(dim + level, level), saturated at `cap` + 1.
int64_t sc_term_count(int dim, int level, int64_t cap);

// The level-`level` Smolyak grid of nested Clenshaw-Curtis rules in `dim`
// variables for the uniform probability measure: digits (row-major
// [n][dim], lexicographic order) and weights [n].
void sc_build_grid(int dim, int level, std::vector<int32_t>& digits, std::vector<double>& weights);

// Every term of the combination formula: term(coefficient, multi-index).
void sc_smolyak_terms(int dim, int level, const std::function<void(double, const std::vector<int>&)>& term);

// Sparse-grid interpolation in the local variables (levels 0..SGI_LEVEL_MAX).
constexpr int SGI_LEVEL_MAX = 5;  // 33 nodes per variable at most
constexpr int SGI_BATCH = 4;      // combination entries evaluated together (entry arrays padded by 3)
struct SgiApplyArgs {
  int32_t ne;  // entries per table row and per S: 10 (symmetric) or 16 (Petrov-Galerkin); 0 = 10
  int32_t npatch, nxi, level, nb, kmax;
  int64_t nsamples;
  double lo, hi;
  const double* table;        // [rows][10]
  const int64_t* off;         // [npatch + 1]
  const int32_t* lv;          // [npatch][4]
  const int32_t* nlv;         // [npatch]
  const double* nodes;        // [nb]: level-i nodes at lofs[i] ...
  int32_t lofs[SGI_LEVEL_MAX + 3];
  int32_t rofs[6];            // row starts of k local variables: cb_rows[rofs[k] .. rofs[k+1]-1]
  const double* cb_coef;      // [entries], grouped by table row
  const uint32_t* cb_boff;    // [entries]: basis offset of variable d in bits 8d..8d+7
  const int32_t* cb_rows;     // per k: npts_k + 1 entry offsets (entries of row r: [r], [r+1])
  const double* xi;           // [nsamples][nxi]
  double* S;                  // [nsamples][npatch][10]
  int32_t* status;            // [nsamples][npatch] or null
  int64_t* list;
  unsigned long long* list_count;
};
size_t sgi_lds_bytes(int kmax, int nb, int level, int ne);
hipError_t launch_sgi_apply(const SgiApplyArgs& a, hipStream_t st);

struct ScApplyArgs {
  int32_t npatch, nxi, D;
  int64_t npoints;
  const int32_t* digits;  // [npoints][nxi]
  const int32_t* lv;      // [npatch][4], -1 padded
  const int32_t* nlv;     // [npatch]
  const int64_t* off;     // [npatch + 1]
  const int64_t* keys;    // [rows], increasing within each patch
  const double* table;    // [rows][10]
  double* S;              // [npoints][npatch][10]
  int32_t* status;        // [npoints][npatch] or null
};

hipError_t launch_sc_apply(const ScApplyArgs& a, hipStream_t st);

// Weighted sums over points: mean[i] = sum_p w_p U[p][i],
// var[i] = sum_p w_p U[p][i]^2 - mean[i]^2; work holds
// sc_quad_work_doubles(npoints, nu) doubles.
int64_t sc_quad_work_doubles(int64_t npoints, int nu);
hipError_t launch_sc_quadrature(const double* U, const double* w, int64_t npoints, int nu, double* mean, double* var,
                                double* work, hipStream_t st);

}  // namespace stomsfem
