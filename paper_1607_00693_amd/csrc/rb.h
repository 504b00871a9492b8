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
  // oversampled patches (launch_rb_os_apply_mfma only): oversampling os_o,
  // corner values Pc [M][4][RBO_NF]; G32 is then the table GO32
  int32_t os_o;
  const double* Pc;
};

hipError_t launch_cell_phi(const UpArgs& args, int a_dtype, double* phi, hipStream_t st);
size_t cell_phi_lds_bytes(int m);
// LDS of one workgroup on gfx950: the FP64 snapshot kernel serves m <= 26
constexpr size_t CELL_PHI_LDS_MAX = 160 * 1024;
// Snapshots of cells beyond the LDS kernels (m <= 64): one wavefront per
// pair, a circular band window in LDS and a global row store of
// cell_phi_band_ws_doubles(m) doubles per workgroup; blocks = workgroups
// (at most npairs), ws holds blocks of them.
hipError_t launch_cell_phi_band(const UpArgs& args, int a_dtype, double* phi, double* ws, int64_t blocks,
                                hipStream_t st);
int64_t cell_phi_band_ws_doubles(int m);
hipError_t launch_rb_build(const RbBuildArgs& b, hipStream_t st);
// Work doubles of the offline build and whether it takes the dual form (the
// method of snapshots, 3 ntrain < (m-1)^2).
int64_t rb_work_doubles(int ncx, int ncy, int m, int ntrain);
bool rb_dual(int m, int ntrain);
hipError_t launch_rb_apply(const RbApplyArgs& ra, int a_dtype, bool f64, hipStream_t st);
int rb_pad_p(int rmax);
int rb_pad_kd(int m);

}  // namespace stomsfem

namespace stomsfem {

// Reduced basis on oversampled patches.  The patch of element K (side
// Mp = m + 2o, moved inside the domain at the edge) is reduced exactly as a
// plain patch (the build above on the patch blocks); the online table GO of
// patch K then holds, per patch element e, RBO_PO coefficients that make
// every linear quantity of the Petrov-Galerkin stiffness a linear function of
// the patch's coefficient values:
//   [0, NA + 3 rmax)        A and Fh of the patch's reduced system (as in G)
//   [RBO_H, RBO_H + 4 NF)   for e inside K: f_e . K_ref p_e^l', f = phibar^0..2
//                           (with the patch boundary data), zeta_0..rmax-1,
//                           l' = K's bilinear test functions 0..3 (zero for
//                           e outside K)
// and Pc [4][NF] the same fields at K's corners (counter-clockwise).
constexpr int RBO_NF = 11;                 // 3 means + 8 modes
constexpr int RBO_H = 60;                  // 36 (A) + 24 (Fh) for rmax = 8
constexpr int RBO_PO = 112;                // RBO_H + 4 NF = 104, padded to 16
struct RbOsArgs {
  int32_t ncx, ncy, m, o, Mp;  // element side m, oversampling o, patch side Mp
  int32_t rmax, KD, PP, KDo;   // G layout (KD x PP), GO rows KDo
  const int32_t* rK;
  const double* Z;       // [Mc][(Mp-1)^2][rmax]
  const double* phibar;  // [Mc][3][(Mp-1)^2]
  const double* G64;     // [Mc][KD][PP]
  double* GO;            // [Mc][KDo][RBO_PO]
  float* GO32;           // [Mc][KDo][RBO_PO]
  double* Pc;            // [Mc][4][RBO_NF]
};
hipError_t launch_rb_os_embed(const void* a, int a_dtype, int64_t nsamples, int ncx, int ncy, int m, int o,
                              double* out, hipStream_t st);
hipError_t launch_rb_os_tables(const RbOsArgs& t, hipStream_t st);
hipError_t launch_rb_os_apply(const RbOsArgs& t, const UpArgs& up, int a_dtype, hipStream_t st);
// FP32 matrix-core online stage (the GEMM of rb_apply_mfma_kernel over the
// patch, PP = RBO_PO, FP64 solve and recombination per pair).
hipError_t launch_rb_os_apply_mfma(const RbApplyArgs& ra, int a_dtype, hipStream_t st);

}  // namespace stomsfem
