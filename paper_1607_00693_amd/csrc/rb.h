// Internal interface of the reduced-basis kernels (rb.hip) for the host
// side of the ABI.
#pragma once
#include "common.h"

namespace stomsfem {

// Layout of the P per-element coefficients for r_max modes:
//   [0, NA)            A_qq', q <= q', row-major upper triangle of r_max x r_max
//   [NA, NA + 3 r_max) Fh_lq at NA + l*r_max + q
//   [.., +6)           B_ll' in the order 00,01,02,11,12,22
__host__ __device__ inline int rb_na(int rmax) { return rmax * (rmax + 1) / 2; }
__host__ __device__ inline int rb_p(int rmax) { return rb_na(rmax) + 3 * rmax + 6; }
__host__ __device__ inline int rb_aidx(int q, int qp, int rmax) {  // q <= qp
  return q * rmax - q * (q - 1) / 2 + (qp - q);
}

struct RbBuildArgs {
  int32_t ncx, ncy, m, ntrain, rmax;  // rmax: storage width of the mode tables
  int32_t rcap;                        // cap on r requested by the caller (<= rmax)
  double tail_tol;
  const void* a;   // training coefficients [ntrain][ncy*m][ncx*m]
  int32_t a_dtype;
  const double* phi;   // [ntrain][M][3][nI]
  double* work;        // rb_work_doubles(...) doubles
  double* Z;           // [M][nI][rmax]
  double* phibar;      // [M][3][nI]
  double* lambda;      // [M][nI] eigenvalues, descending
  int32_t* rK;         // [M]
  float* G32;          // [M][KD][PP]
  double* G64;         // [M][KD][PP]
  int32_t KD, PP;      // padded element count and padded P
  int32_t max_sweeps;
};

struct RbApplyArgs {
  UpArgs up;
  int32_t rmax, KD, PP;
  const int32_t* rK;
  const float* G32;
  const double* G64;
};

hipError_t launch_cell_phi(const UpArgs& args, int a_dtype, double* phi, hipStream_t st);
size_t cell_phi_lds_bytes(int m);
hipError_t launch_rb_build(const RbBuildArgs& b, hipStream_t st);
// Work doubles of the offline build and whether it takes the dual form (the
// method of snapshots, 3 ntrain < (m-1)^2).
int64_t rb_work_doubles(int ncx, int ncy, int m, int ntrain);
bool rb_dual(int m, int ntrain);
hipError_t launch_rb_apply(const RbApplyArgs& ra, int a_dtype, bool f64, hipStream_t st);
int rb_pad_p(int rmax);
int rb_pad_kd(int m);

}  // namespace stomsfem
