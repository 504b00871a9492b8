// FP32 factorization with FP64 residual refinement: arguments and launchers
// (kernels in upscale_mixed.hip).
#pragma once
#include "common.h"

namespace stomsfem {

struct MixedArgs {
  UpArgs up;
  double tol;                   // on max_l |r^l|_inf / |f^l|_inf
  int32_t max_iter;             // refinement solves
  int64_t* list;                // pairs handed to the FP64 path
  unsigned long long* count;
};

size_t upscale_mixed_lds_bytes(int m);
hipError_t launch_upscale_mixed(const MixedArgs& a, int a_dtype, hipStream_t st);
hipError_t launch_gather_blocks(const UpArgs& up, int a_dtype, const int64_t* list, int64_t count, double* out,
                                hipStream_t st);

}  // namespace stomsfem
