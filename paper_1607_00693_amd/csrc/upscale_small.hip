// Local upscaling, one (coarse element, sample) pair per lane, for m <= 8.
//
// Cell problems (Sec. 2.2, eq. MsFEM cell problem; Sec. 3 eq. MsFEB2): on the
// m x m fine Q1 grid of a coarse element K, with interior unknowns x_I and
// boundary data g^l = p^l,
//     K_II x_I^l = f^l := -K_IB g^l ,      l = 0, 1, 2,
// and the upscaled stiffness (eq. stiffness_local) is the Schur complement
// of the local stiffness onto the boundary, contracted with the data:
//     S_ll' = g^l . K_BB g^l'  -  f^l . K_II^{-1} f^l' .
// With K_II = L D L^T (unit lower L, natural node order, half-bandwidth m)
// and y^l = L^{-1} f^l, the second term is sum_j y_j^l y_j^l' / d_j, so the
// factor is consumed as it is produced: a sliding (m+1) x (m+1) window of
// the band is all that is ever stored, and no back substitution is needed.
// phi^3 = 1 - sum phi^l gives the fourth row and column (S 1 = 0).
//
// Everything here is compile-time structured: the loop over the NI = (m-1)^2
// pivots is fully unrolled, the window lives in registers with static
// indices, and only the coefficient values are runtime data.  The
// coefficient block is read row by row (two element rows live at a time).
#include "small_cell.h"

namespace stomsfem {

template <int M, typename T, int BS>
__global__ __launch_bounds__(BS) void upscale_lane_kernel(UpArgs args) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= args.npairs) return;
  const int Mc = args.ncx * args.ncy;
  const int64_t s = p / Mc;
  const int K = (int)(p - s * Mc);
  SmallCell<M, T> cell;
  cell.a = (const T*)args.a + block_offset(s, K, args.ncx, args.ncy, M);
  cell.lda = (int64_t)args.ncx * M;
  cell.run(args.S + p * 10, args.status ? args.status + p : nullptr);
}

template <int M, typename T, int BS>
static hipError_t launch_lane_bs(const UpArgs& args, hipStream_t st) {
  const int64_t blocks = (args.npairs + BS - 1) / BS;
  hipLaunchKernelGGL((upscale_lane_kernel<M, T, BS>), dim3((unsigned)blocks), dim3(BS), 0, st, args);
  return hipGetLastError();
}

template <int M, typename T>
static hipError_t launch_lane(const UpArgs& args, int block, hipStream_t st) {
  if (block == 128) return launch_lane_bs<M, T, 128>(args, st);
  if (block == 256) return launch_lane_bs<M, T, 256>(args, st);
  return launch_lane_bs<M, T, 64>(args, st);
}

hipError_t launch_upscale_small(const UpArgs& args, int a_dtype, hipStream_t st, int block) {
  const bool f32 = a_dtype == STOMSFEM_F32;
#define CASE(MM)                                                                           \
  case MM:                                                                                 \
    return f32 ? launch_lane<MM, float>(args, block, st) : launch_lane<MM, double>(args, block, st);
  switch (args.m) {
    CASE(1)
    CASE(2)
    CASE(3)
    CASE(4)
    CASE(5)
    CASE(6)
    CASE(7)
    CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef CASE
}

}  // namespace stomsfem
