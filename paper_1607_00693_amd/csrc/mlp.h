// Internal interface of the surrogate kernels (mlp.hip).
#pragma once
#include "common.h"

namespace stomsfem {

constexpr int MLP_KIN = 4;     // local variables (zero padded)
constexpr int MLP_WIDTH = 64;
constexpr int MLP_NOUT2 = 20;  // two heads x 10 entries
constexpr int MLP_BATCH = 32;  // training minibatch
// parameter packing (floats, per patch)
constexpr int MLP_OW1 = 0;
constexpr int MLP_OB1 = MLP_OW1 + MLP_KIN * MLP_WIDTH;
constexpr int MLP_OW2 = MLP_OB1 + MLP_WIDTH;
constexpr int MLP_OB2 = MLP_OW2 + MLP_WIDTH * MLP_WIDTH;
constexpr int MLP_OW3 = MLP_OB2 + MLP_WIDTH;
constexpr int MLP_OB3 = MLP_OW3 + MLP_WIDTH * MLP_WIDTH;
constexpr int MLP_OW4 = MLP_OB3 + MLP_WIDTH;
constexpr int MLP_OB4 = MLP_OW4 + MLP_WIDTH * MLP_NOUT2;
constexpr int MLP_NP = MLP_OB4 + MLP_NOUT2;
// per-pair status of the surrogate stage
constexpr int MLP_ST_ACCEPTED = 0;
constexpr int MLP_ST_FALLBACK = 1;
constexpr int MLP_ST_AUDIT = 2;

struct MlpTrainArgs {
  int32_t npatch;
  int64_t ntrain;
  int32_t steps;
  int64_t t0;           // Adam steps already taken
  float lr;
  float* params;        // [M][NP]
  float* m1;            // [M][NP] (training)
  float* m2;
  const float* X;       // [M][ntrain][KIN]
  const float* T;       // [M][ntrain][10]
  const int64_t* perm;  // [ntrain] minibatch order, or NULL for identity
  const float* xb;      // gradient mode: [M][BATCH][KIN] batch, else NULL
  const float* tb;      // gradient mode: [M][BATCH][10]
  float* grads;         // gradient mode: [M][NP]
  float* loss;          // [M] loss of the last minibatch, or NULL
};

// Coefficient family of a surrogate: 0 = the bump family (inputs xi_j as
// they are); 1 = the channels-and-inclusions medium: inputs 2 sigmoid(xi_j) - 1
// (the fraction of the conductivity decades, in [-1, 1]) and outputs S divided
// by the mean conductivity over the patch's boundary ring of fine elements,
// 1 + sum_c rw_c (theta_c - 1) with rw_c the fraction of ring elements owned
// by local feature c (with linear boundary conditions the boundary elements
// carry the prescribed gradient, so this mean follows max|S| over the decades
// far more closely than the patch mean does); a patch with more than four
// local features carries the local-variable sentinel -2 and always takes the
// plain path.
constexpr int MLP_FAMILY_BUMPS = 0;
constexpr int MLP_FAMILY_FEATURES = 1;
constexpr int MLP_LV_ALWAYS_PLAIN = -2;

struct MlpDataArgs {
  int32_t family;
  double decades;
  const double* rw;     // family 1: [M][KIN] ring fractions of the local features
  int32_t npatch, nxi;
  int64_t ntrain;
  const int32_t* lv;    // [M][KIN]
  const double* xi;     // [ntrain][nxi]
  const double* S;      // [ntrain][M][10]
  double* mu;           // [M][10]
  double* sd;           // [M][10]
  double* sd_raw;       // [M][10] scratch
  float* X;             // [M][ntrain][KIN]
  float* T;             // [M][ntrain][10]
};

struct MlpInferArgs {
  int32_t family;
  double decades;
  const double* rw;     // family 1: [M][KIN] ring fractions of the local features
  int32_t npatch, ncx, nxi;
  int64_t nsamples;
  const float* params;
  const int32_t* lv;
  const double* mu;
  const double* sd;
  const double* xi;     // [nsamples][nxi]
  double box, tau;
  float* Y;             // raw outputs [nsamples][M][20], or NULL
  double* S;            // [nsamples][M][10], or NULL (prediction only)
  int32_t* status;      // [nsamples][M], or NULL
  unsigned long long* count;  // device counter of listed pairs
  int64_t* list;        // [nsamples*M] pairs for the plain solve
  unsigned long long* stats;  // [4] or NULL
  int32_t bump_g;
  double bump_rho, bump_eps, bump_base, bump_amp, bump_beta;
  int32_t m;            // fine cells per patch side; the fused fallback serves m = 8
  double* gate;         // [nsamples][M][2] residual and uncertainty of the gate, or NULL
};

hipError_t launch_mlp_train(const MlpTrainArgs& a, bool train, hipStream_t st);
hipError_t launch_mlp_data(const MlpDataArgs& d, hipStream_t st);
// Inference variants: FP32 reference, BF16 matrix cores with three-term
// splitting, FP16 matrix cores with single terms.
constexpr int MLP_MODE_F32 = 0;
constexpr int MLP_MODE_BF16 = 1;
constexpr int MLP_MODE_F16 = 2;
hipError_t launch_mlp_infer(const MlpInferArgs& a, int mode, hipStream_t st);
// The gate alone on given raw outputs Y [nsamples][M][20] (a.S, a.status,
// a.gate written; no audit, no fallback).
hipError_t launch_mlp_gate(const MlpInferArgs& a, const float* Y, hipStream_t st);
// Second half of the plain fallback for m != 8: the listed pairs' plain S
// (Sc, stc, computed by the regular kernels on regenerated coefficients) is
// compared with the prediction in S, stored, and counted as the fused
// fallback does.
hipError_t launch_mlp_fallback_finish(const int64_t* list, int64_t count, const double* Sc, const int32_t* stc,
                                      double* S, int32_t* status, unsigned long long* stats, hipStream_t st);

}  // namespace stomsfem
