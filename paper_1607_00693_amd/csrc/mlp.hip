// Learned per-patch surrogate for the upscaled stiffness.
//
// Per coarse element K: local random variables x (the xi_j whose mode
// touches K, Sec. 3 eq. MsFEB2, zero padded to 4) -> 64 -> 64 -> 64 -> 2 x 10,
// GELU (exact erf form), two output heads predicting the standardised 10
// unique entries of S_K.  Trained on pairs produced by the plain path.
//
//   mlp_train_kernel<TRAIN>  FP32 forward / hand-written backward over a
//                            minibatch of 32, one workgroup per patch; with
//                            TRAIN the Adam update is applied to each
//                            parameter by the thread that formed its
//                            gradient, otherwise the raw gradient is written
//                            (parity checks against the oracle).
//   mlp_infer_mma_kernel<F16> matrix-core inference (FP32 accumulation,
//                            activations kept in registers, tabulated GELU),
//                            then the gate per pair: BF16 with three-term
//                            splitting of weights and activations
//                            (v_mfma_f32_16x16x32_bf16), or FP16 single
//                            terms (v_mfma_f32_16x16x32_f16);
//   mlp_infer_f32_kernel     FP32 inference (reference for the BF16 one);
//   mlp_fallback_kernel      plain solve (m = 8 lane kernel) of the pairs the
//                            gate rejected plus a 1% audit of accepted ones,
//                            with the coefficients regenerated from xi.
//
// Gate: S = (S_A + S_B)/2 of the de-standardised heads; residual =
// max_l |sum_l' S_ll'| / max|S| (every exact S has zero row sums) and
// uncertainty = max|S_A - S_B| / max|S|; accepted when both are <= tau and
// every local variable lies in the training box; accepted S are projected
// onto the zero-row-sum matrices, S <- P S P, P = I - 1 1^T / 4.
#include "mlp.h"
#include "small_cell.h"

namespace stomsfem {


__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float Phi = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float phi = expf(-0.5f * z * z) * 0.39894228040143268f;
  return Phi + z * phi;
}

// network input of local variable value xi, and the output scale of a
// (sample, patch): see MLP_FAMILY_FEATURES
__device__ __forceinline__ double mlp_input(int family, double xi) {
  return family == MLP_FAMILY_FEATURES ? 2.0 / (1.0 + exp(-xi)) - 1.0 : xi;
}
__device__ __forceinline__ double mlp_out_scale(int family, double decades, const int32_t* lv, const double* rw,
                                                const double* xs) {
  if (family != MLP_FAMILY_FEATURES) return 1.0;
  double sc = 1.0;
  for (int c = 0; c < MLP_KIN; ++c)
    if (lv[c] >= 0) sc += rw[c] * (feature_theta(xs[lv[c]], decades) - 1.0);
  return sc;
}

// ---------------------------------------------------------------------------
// Training / gradients
// ---------------------------------------------------------------------------
constexpr int MB = MLP_BATCH;  // minibatch per step
constexpr int WD = MLP_WIDTH;
constexpr int NO = MLP_NOUT2;

template <bool TRAIN>
__global__ __launch_bounds__(256) void mlp_train_kernel(MlpTrainArgs a) {
  const int K = blockIdx.x;
  const int tid = threadIdx.x;
  float* P = a.params + (int64_t)K * MLP_NP;
  float* m1 = a.m1 ? a.m1 + (int64_t)K * MLP_NP : nullptr;
  float* m2 = a.m2 ? a.m2 + (int64_t)K * MLP_NP : nullptr;
  __shared__ float X[MB][MLP_KIN], Tg[MB][10];
  __shared__ float H1[MB][WD], G1[MB][WD], H2[MB][WD], G2[MB][WD], H3[MB][WD], G3[MB][WD], D[MB][WD];
  __shared__ float dY[MB][NO];
  __shared__ float red[256];
  float* W1 = P + MLP_OW1;
  float* b1 = P + MLP_OB1;
  float* W2 = P + MLP_OW2;
  float* b2 = P + MLP_OB2;
  float* W3 = P + MLP_OW3;
  float* b3 = P + MLP_OB3;
  float* W4 = P + MLP_OW4;
  float* b4 = P + MLP_OB4;
  const float bc1 = 0.9f, bc2 = 0.999f;

  for (int step = 0; step < a.steps; ++step) {
    const int64_t t = a.t0 + step + 1;  // Adam step count
    const float corr1 = 1.0f - powf(bc1, (float)t), corr2 = 1.0f - powf(bc2, (float)t);
    // minibatch
    for (int i = tid; i < MB * (MLP_KIN + 10); i += 256) {
      const int b = i / (MLP_KIN + 10), c = i % (MLP_KIN + 10);
      int64_t idx;
      if (a.xb) {
        idx = b;
      } else {
        const int64_t pos = ((int64_t)(a.t0 + step) * MB + b) % a.ntrain;
        idx = a.perm ? a.perm[pos] : pos;
        idx = idx < 0 ? 0 : (idx >= a.ntrain ? a.ntrain - 1 : idx);  // a malformed perm cannot read out of bounds
      }
      if (c < MLP_KIN) {
        X[b][c] = a.xb ? a.xb[((int64_t)K * MB + b) * MLP_KIN + c] : a.X[((int64_t)K * a.ntrain + idx) * MLP_KIN + c];
      } else {
        const int q = c - MLP_KIN;
        Tg[b][q] = a.tb ? a.tb[((int64_t)K * MB + b) * 10 + q] : a.T[((int64_t)K * a.ntrain + idx) * 10 + q];
      }
    }
    __syncthreads();
    // forward
    for (int i = tid; i < MB * WD; i += 256) {
      const int b = i / WD, j = i % WD;
      float z = b1[j];
#pragma unroll
      for (int k = 0; k < MLP_KIN; ++k) z += X[b][k] * W1[k * WD + j];
      H1[b][j] = gelu_f(z);
      G1[b][j] = gelu_grad_f(z);
    }
    __syncthreads();
    for (int i = tid; i < MB * WD; i += 256) {
      const int b = i / WD, j = i % WD;
      float z = b2[j];
      for (int k = 0; k < WD; ++k) z += H1[b][k] * W2[k * WD + j];
      H2[b][j] = gelu_f(z);
      G2[b][j] = gelu_grad_f(z);
    }
    __syncthreads();
    for (int i = tid; i < MB * WD; i += 256) {
      const int b = i / WD, j = i % WD;
      float z = b3[j];
      for (int k = 0; k < WD; ++k) z += H2[b][k] * W3[k * WD + j];
      H3[b][j] = gelu_f(z);
      G3[b][j] = gelu_grad_f(z);
    }
    __syncthreads();
    float lpart = 0.0f;
    for (int i = tid; i < MB * NO; i += 256) {
      const int b = i / NO, o = i % NO;
      float y = b4[o];
      for (int k = 0; k < WD; ++k) y += H3[b][k] * W4[k * NO + o];
      const float r = y - Tg[b][o % 10];
      lpart += r * r;
      dY[b][o] = 2.0f * r / (float)(MB * NO);
    }
    red[tid] = lpart;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0 && a.loss) a.loss[K] = red[0] / (float)(MB * NO);
    // backward; each parameter's gradient is formed by one thread
    auto apply = [&](float* /*base*/, int idx, float gval) {
      if (TRAIN) {
        const float mm1 = bc1 * m1[idx] + (1.0f - bc1) * gval;
        const float mm2 = bc2 * m2[idx] + (1.0f - bc2) * gval * gval;
        m1[idx] = mm1;
        m2[idx] = mm2;
        P[idx] -= a.lr * (mm1 / corr1) / (sqrtf(mm2 / corr2) + 1e-8f);
      } else {
        a.grads[(int64_t)K * MLP_NP + idx] = gval;
      }
    };
    // dZ3 = (dY W4^T) .* gelu'(Z3)
    for (int i = tid; i < MB * WD; i += 256) {
      const int b = i / WD, j = i % WD;
      float s = 0.0f;
      for (int o = 0; o < NO; ++o) s += dY[b][o] * W4[j * NO + o];
      D[b][j] = s * G3[b][j];
    }
    __syncthreads();
    for (int i = tid; i < WD * NO + NO; i += 256) {
      float gval = 0.0f;
      if (i < WD * NO) {
        const int k = i / NO, o = i % NO;
        for (int b = 0; b < MB; ++b) gval += H3[b][k] * dY[b][o];
        apply(P, MLP_OW4 + i, gval);
      } else {
        const int o = i - WD * NO;
        for (int b = 0; b < MB; ++b) gval += dY[b][o];
        apply(P, MLP_OB4 + o, gval);
      }
    }
    __syncthreads();
    // dZ2 = (dZ3 W3^T) .* gelu'(Z2)  -> stored in G3 (no longer needed)
    for (int i = tid; i < MB * WD; i += 256) {
      const int b = i / WD, j = i % WD;
      float s = 0.0f;
      for (int o = 0; o < WD; ++o) s += D[b][o] * W3[j * WD + o];
      G3[b][j] = s * G2[b][j];
    }
    __syncthreads();
    for (int i = tid; i < WD * WD + WD; i += 256) {
      float gval = 0.0f;
      if (i < WD * WD) {
        const int k = i / WD, o = i % WD;
        for (int b = 0; b < MB; ++b) gval += H2[b][k] * D[b][o];
        apply(P, MLP_OW3 + i, gval);
      } else {
        const int o = i - WD * WD;
        for (int b = 0; b < MB; ++b) gval += D[b][o];
        apply(P, MLP_OB3 + o, gval);
      }
    }
    __syncthreads();
    // dZ1 = (dZ2 W2^T) .* gelu'(Z1)  -> stored in D
    for (int i = tid; i < MB * WD; i += 256) {
      const int b = i / WD, j = i % WD;
      float s = 0.0f;
      for (int o = 0; o < WD; ++o) s += G3[b][o] * W2[j * WD + o];
      D[b][j] = s * G1[b][j];
    }
    __syncthreads();
    for (int i = tid; i < WD * WD + WD; i += 256) {
      float gval = 0.0f;
      if (i < WD * WD) {
        const int k = i / WD, o = i % WD;
        for (int b = 0; b < MB; ++b) gval += H1[b][k] * G3[b][o];
        apply(P, MLP_OW2 + i, gval);
      } else {
        const int o = i - WD * WD;
        for (int b = 0; b < MB; ++b) gval += G3[b][o];
        apply(P, MLP_OB2 + o, gval);
      }
    }
    for (int i = tid; i < MLP_KIN * WD + WD; i += 256) {
      float gval = 0.0f;
      if (i < MLP_KIN * WD) {
        const int k = i / WD, o = i % WD;
        for (int b = 0; b < MB; ++b) gval += X[b][k] * D[b][o];
        apply(P, MLP_OW1 + i, gval);
      } else {
        const int o = i - MLP_KIN * WD;
        for (int b = 0; b < MB; ++b) gval += D[b][o];
        apply(P, MLP_OB1 + o, gval);
      }
    }
    __syncthreads();
  }
}

hipError_t launch_mlp_train(const MlpTrainArgs& a, bool train, hipStream_t st) {
  if (train)
    hipLaunchKernelGGL(mlp_train_kernel<true>, dim3(a.npatch), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(mlp_train_kernel<false>, dim3(a.npatch), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Gather the local variables and standardised targets of the training set.
__global__ void mlp_gather_kernel(MlpDataArgs d) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)d.npatch * d.ntrain;
  if (t >= total) return;
  const int K = (int)(t / d.ntrain);
  const int64_t s = t % d.ntrain;
  for (int c = 0; c < MLP_KIN; ++c) {
    const int j = d.lv[K * MLP_KIN + c];
    d.X[t * MLP_KIN + c] = j >= 0 ? (float)mlp_input(d.family, d.xi[s * d.nxi + j]) : 0.0f;
  }
  const double* S = d.S + (s * d.npatch + K) * 10;
  const double sc = mlp_out_scale(d.family, d.decades, d.lv + K * MLP_KIN, d.rw + K * MLP_KIN, d.xi + s * d.nxi);
  for (int q = 0; q < 10; ++q) d.T[t * 10 + q] = (float)((S[q] / sc - d.mu[K * 10 + q]) / d.sd[K * 10 + q]);
}

// Per-patch, per-entry mean and standard deviation (FP64, fixed order).
__global__ void mlp_stats_kernel(MlpDataArgs d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.npatch * 10) return;
  const int K = t / 10, q = t % 10;
  const int32_t* lv = d.lv + K * MLP_KIN;
  const double* rw = d.rw + K * MLP_KIN;
  double m = 0.0;
  for (int64_t s = 0; s < d.ntrain; ++s)
    m += d.S[(s * d.npatch + K) * 10 + q] / mlp_out_scale(d.family, d.decades, lv, rw, d.xi + s * d.nxi);
  m /= (double)d.ntrain;
  double v = 0.0;
  for (int64_t s = 0; s < d.ntrain; ++s) {
    const double e = d.S[(s * d.npatch + K) * 10 + q] / mlp_out_scale(d.family, d.decades, lv, rw, d.xi + s * d.nxi) - m;
    v += e * e;
  }
  double sd = sqrt(v / (double)d.ntrain);
  d.mu[t] = m;
  d.sd_raw[t] = sd;
}

__global__ void mlp_stats_floor_kernel(MlpDataArgs d) {
  const int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= d.npatch) return;
  double mx = 1.0;
  for (int q = 0; q < 10; ++q) mx = fmax(mx, fabs(d.mu[K * 10 + q]));
  for (int q = 0; q < 10; ++q) d.sd[K * 10 + q] = fmax(d.sd_raw[K * 10 + q], 1e-12 * mx);
}

hipError_t launch_mlp_data(const MlpDataArgs& d, hipStream_t st) {
  hipLaunchKernelGGL(mlp_stats_kernel, dim3((d.npatch * 10 + 63) / 64), dim3(64), 0, st, d);
  hipLaunchKernelGGL(mlp_stats_floor_kernel, dim3((d.npatch + 63) / 64), dim3(64), 0, st, d);
  const int64_t total = (int64_t)d.npatch * d.ntrain;
  hipLaunchKernelGGL(mlp_gather_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inference and gate
// ---------------------------------------------------------------------------
// The gate of one pair from its 20 raw outputs y (heads A and B, each
// de-standardised and multiplied by the output scale osc): writes the
// stored S (P S P if accepted, else the head mean), the residual and the
// uncertainty, and returns acceptance.  A pair is accepted only if all 20
// de-standardised values are finite, max|S| > 0, both signals are <= tau and
// every local variable is inside the box; with a non-finite value the two
// signals are NaN (comparisons are written so that NaN never passes).
__device__ __forceinline__ bool gate_pair(const double* __restrict__ mu, const double* __restrict__ sd,
                                          const float* y, double osc, bool inbox, double tau, double* Sout,
                                          double* resid_out, double* unc_out) {
  double SA[10], SB[10], S[10];
  double scale = 0.0, unc = 0.0;
  bool finite = true;
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    SA[q] = osc * (mu[q] + sd[q] * (double)y[q]);
    SB[q] = osc * (mu[q] + sd[q] * (double)y[10 + q]);
    finite = finite && isfinite(SA[q]) && isfinite(SB[q]);
    S[q] = 0.5 * (SA[q] + SB[q]);
    scale = fmax(scale, fabs(S[q]));
    unc = fmax(unc, fabs(SA[q] - SB[q]));
  }
  // unpack (00,01,02,03,11,12,13,22,23,33)
  const double s4[4][4] = {{S[0], S[1], S[2], S[3]}, {S[1], S[4], S[5], S[6]}, {S[2], S[5], S[7], S[8]},
                           {S[3], S[6], S[8], S[9]}};
  double resid = 0.0, rs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    rs[i] = (s4[i][0] + s4[i][1]) + (s4[i][2] + s4[i][3]);
    resid = fmax(resid, fabs(rs[i]));
  }
  const double tol = tau * scale;
  const bool ok = finite && inbox && scale > 0.0 && resid <= tol && unc <= tol;
  // P S P with P = I - 1 1^T / 4
  const double tot = (rs[0] + rs[1]) + (rs[2] + rs[3]);
  double pr[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) pr[i][j] = s4[i][j] - 0.25 * rs[i] - 0.25 * rs[j] + 0.0625 * tot;
  const double outv[10] = {pr[0][0], pr[0][1], pr[0][2], pr[0][3], pr[1][1],
                           pr[1][2], pr[1][3], pr[2][2], pr[2][3], pr[3][3]};
#pragma unroll
  for (int q = 0; q < 10; ++q) Sout[q] = ok ? outv[q] : S[q];
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  *resid_out = finite && scale > 0.0 ? resid / scale : nan;
  *unc_out = finite && scale > 0.0 ? unc / scale : nan;
  return ok;
}

__device__ __forceinline__ bool local_vars_in_box(const MlpInferArgs& a, int K, int64_t s) {
  bool inbox = true;
  for (int c = 0; c < MLP_KIN; ++c) {
    const int j = a.lv[K * MLP_KIN + c];
    if (j == MLP_LV_ALWAYS_PLAIN) inbox = false;
    if (j >= 0 && !(fabs(a.xi[s * a.nxi + j]) <= a.box)) inbox = false;
  }
  return inbox;
}

__device__ __forceinline__ double out_scale_of(const MlpInferArgs& a, int K, int64_t s) {
  return mlp_out_scale(a.family, a.decades, a.lv + K * MLP_KIN, a.rw + K * MLP_KIN, a.xi + s * a.nxi);
}

__device__ __forceinline__ void gate_and_store(const MlpInferArgs& a, int K, int64_t s, const float* y, double* Sout,
                                               int32_t* st, bool* fallback) {
  const int64_t p = s * a.npatch + K;
  double resid, unc;
  const bool ok = gate_pair(a.mu + K * 10, a.sd + K * 10, y, out_scale_of(a, K, s), local_vars_in_box(a, K, s), a.tau,
                            Sout, &resid, &unc);
  if (a.gate) {
    a.gate[2 * p] = resid;
    a.gate[2 * p + 1] = unc;
  }
  const bool audit = ok && ((uint64_t)p * 2654435761ull) % 100ull == 0ull;
  if (st) *st = ok ? (audit ? MLP_ST_AUDIT : MLP_ST_ACCEPTED) : MLP_ST_FALLBACK;
  *fallback = !ok || audit;
}

// The gate alone on given raw outputs Y [nsamples][M][20]: one thread per
// pair; status 0 = accepted, 1 = rejected (no audit, no fallback).
__global__ __launch_bounds__(256) void mlp_gate_kernel(MlpInferArgs a, const float* __restrict__ Yin) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= a.nsamples * a.npatch) return;
  const int64_t s = p / a.npatch;
  const int K = (int)(p - s * a.npatch);
  float y[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) y[o] = Yin[p * NO + o];
  double resid, unc;
  const bool ok = gate_pair(a.mu + K * 10, a.sd + K * 10, y, out_scale_of(a, K, s), local_vars_in_box(a, K, s), a.tau,
                            a.S + p * 10, &resid, &unc);
  if (a.gate) {
    a.gate[2 * p] = resid;
    a.gate[2 * p + 1] = unc;
  }
  if (a.status) a.status[p] = ok ? MLP_ST_ACCEPTED : MLP_ST_FALLBACK;
}

hipError_t launch_mlp_gate(const MlpInferArgs& a, const float* Y, hipStream_t st) {
  const int64_t n = a.nsamples * a.npatch;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_gate_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, Y);
  return hipGetLastError();
}

__device__ __forceinline__ void push_fallback(const MlpInferArgs& a, int64_t p) {
  const unsigned long long idx = atomicAdd((unsigned long long*)a.count, 1ull);
  a.list[idx] = p;
}

// FP32 reference inference: one lane per pair, weights of the patch and each
// lane's hidden activations in LDS.
__global__ __launch_bounds__(64) void mlp_infer_f32_kernel(MlpInferArgs a) {
  const int K = blockIdx.y;
  __shared__ float Wl[MLP_NP];
  __shared__ float Hl[64][WD + 1];
  const float* P = a.params + (int64_t)K * MLP_NP;
  for (int i = threadIdx.x; i < MLP_NP; i += 64) Wl[i] = P[i];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (s >= a.nsamples) return;
  float* h = Hl[threadIdx.x];
  float x[MLP_KIN], z[WD];
#pragma unroll
  for (int c = 0; c < MLP_KIN; ++c) {
    const int j = a.lv[K * MLP_KIN + c];
    x[c] = j >= 0 ? (float)mlp_input(a.family, a.xi[s * a.nxi + j]) : 0.0f;
  }
#pragma unroll
  for (int j = 0; j < WD; ++j) z[j] = Wl[MLP_OB1 + j];
#pragma unroll
  for (int k = 0; k < MLP_KIN; ++k)
#pragma unroll
    for (int j = 0; j < WD; ++j) z[j] += x[k] * Wl[MLP_OW1 + k * WD + j];
#pragma unroll
  for (int j = 0; j < WD; ++j) h[j] = gelu_f(z[j]);
  for (int L = 0; L < 2; ++L) {
    const int ob = L == 0 ? MLP_OB2 : MLP_OB3, ow = L == 0 ? MLP_OW2 : MLP_OW3;
#pragma unroll
    for (int j = 0; j < WD; ++j) z[j] = Wl[ob + j];
    for (int k = 0; k < WD; ++k) {
      const float hk = h[k];
#pragma unroll
      for (int j = 0; j < WD; ++j) z[j] += hk * Wl[ow + k * WD + j];
    }
#pragma unroll
    for (int j = 0; j < WD; ++j) h[j] = gelu_f(z[j]);
  }
  float y[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) y[o] = Wl[MLP_OB4 + o];
  for (int k = 0; k < WD; ++k) {
    const float hk = h[k];
#pragma unroll
    for (int o = 0; o < NO; ++o) y[o] += hk * Wl[MLP_OW4 + k * NO + o];
  }
  const int64_t p = s * a.npatch + K;
  if (a.Y) {
    for (int o = 0; o < NO; ++o) a.Y[p * NO + o] = y[o];
  }
  if (a.S) {
    bool fb;
    gate_and_store(a, K, s, y, a.S + p * 10, a.status ? a.status + p : nullptr, &fb);
    if (fb) push_fallback(a, p);
  }
}

// Matrix-core inference, BF16 (v_mfma_f32_16x16x32_bf16) or FP16
// (v_mfma_f32_16x16x32_f16), FP32 accumulation.
//
// Every FP32 weight w and activation h is carried as two bf16 numbers,
// w = w_hi + w_lo, h = h_hi + h_lo (w_hi = bf16(w), w_lo = bf16(w - w_hi)), and
// each product is formed as h_hi w_hi + h_hi w_lo + h_lo w_hi on the matrix
// cores (the h_lo w_lo term is below 2^-16 relative), which keeps the layers
// at about 16 significant bits.  The FP16 variant carries every value as one
// fp16 number and forms one product: its 11-bit significand (bf16 has 8) is
// enough for the gate to accept as many pairs as with the three-term BF16
// form on the trained networks, at a third of the matrix work, half the
// operand registers and LDS (two workgroups per CU) and no splitting.
//
// The layers are computed transposed, D = W^T H^T (rows = output neurons,
// columns = 16 samples), so that the accumulator layout of one layer is the
// B-operand layout of the next: for a 16 x 16 output tile, lane l holds
// neurons 4(l/16) + v (v < 4) of sample l % 16; for a 32-wide k block the
// B operand wants 8 k values of sample l % 16 in lane l, and the two output
// tiles 2kb and 2kb+1 supply exactly 8 such values per lane.  The k order
// inside the block is therefore a permutation (slot 8g + j holds neuron
// 32kb + 4g + j for j < 4 and 32kb + 16 + 4g + (j - 4) otherwise, g = l / 16),
// and the weights are staged once per workgroup in LDS in that permuted A
// layout (16 bytes per lane and operand, one ds_read_b128).  Activations never
// leave the registers; biases initialise the accumulators.
//
// GELU: Phi(z) interpolated linearly in an LDS table built by every
// workgroup (gelu_lin: nodes 1/256 apart for BF16, 1/128 for FP16).  The erf
// form is evaluated exactly by the FP32 reference kernel and the training
// kernel.
//
// Workgroup = 8 wavefronts on one patch; a wavefront takes 64 samples (four
// column tiles of 16, in one pass for BF16 and two for FP16), parks the 20
// outputs of each sample in LDS and then
// gates one sample per lane; rejected and audited pairs are appended to the
// fallback list with one atomic per wavefront.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int BF_WAVES = 8;                 // wavefronts per workgroup
constexpr int BF_TILE = 64 * BF_WAVES;      // samples per workgroup tile
constexpr int BF_NOP = 32;                  // 20 outputs padded to two row tiles
// A operands: layer 1 (4 row tiles x 1 k block), layers 2 and 3 (4 x 2),
// layer 4 (2 x 2); each x {hi, lo} x 64 lanes x 8 bf16
constexpr int BF_OPS_L1 = 0, BF_OPS_L2 = 4, BF_OPS_L3 = 12, BF_OPS_L4 = 20, BF_OPS = 24;

// GELU of the matrix-core kernels: Phi linear between nodes on [-6, 6] (value
// and increment at each node, one 8-byte table read per activation; Phi from
// the FP64 erfc at the nodes, 0 or 1 to FP32 precision outside the range).
// FP16 variant: nodes 1/128 apart, interpolation error below 2e-6 in Phi, so
// below 1.2e-5 in gelu(z) for |z| <= 6, far under the fp16 rounding
// (2^-11 relative) the activations then take; 12 KB.
// The BF16 variant, whose layers carry about 16 significant bits, uses
// nodes 1/256 apart (error below 5e-7 in Phi, 3e-6 in gelu(z)) in 24 KB.
template <bool F16>
struct GeluLin {
  static constexpr int N = F16 ? 1536 : 3072;  // intervals on [-6, 6]
  static constexpr float SCALE = F16 ? 128.0f : 256.0f, OFF = 6.0f * SCALE;
};
template <bool F16>
__device__ __forceinline__ float gelu_lin(const float2* __restrict__ tab, float z) {
  using G = GeluLin<F16>;
  float u = fmaf(z, G::SCALE, G::OFF);
  u = fminf(fmaxf(u, 0.0f), (float)G::N - 0.0009765625f);
  const int i = (int)u;
  const float t = __builtin_amdgcn_fractf(u);
  const float2 c = tab[i];
  return z * fmaf(t, c.y, c.x);
}


// split four consecutive activations of two tiles into hi/lo B operands
__device__ __forceinline__ void split8(const f32x4_t& a, const f32x4_t& b, bf16x8_t& hi, bf16x8_t& lo) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const __bf16 ha = (__bf16)a[v], hb = (__bf16)b[v];
    hi[v] = ha;
    hi[4 + v] = hb;
    lo[v] = (__bf16)(a[v] - (float)ha);
    lo[4 + v] = (__bf16)(b[v] - (float)hb);
  }
}

__device__ __forceinline__ f32x4_t mma3(const bf16x8_t& ah, const bf16x8_t& al, const bf16x8_t& bh,
                                        const bf16x8_t& bl, f32x4_t c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
}

// Orders the LDS accesses of one wavefront across its lanes (a wave barrier
// between release and acquire fences of wavefront scope).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Operand types of the two matrix-core variants: BF16 carries every value as
// hi + lo (two terms, three products), FP16 as one term (one product).
template <bool F16>
struct MmaOps {
  typedef bf16x8_t V;
  static constexpr int NS = 2;  // terms per value
  __device__ static __forceinline__ void split(const f32x4_t& a, const f32x4_t& b, V& hi, V& lo) {
    split8(a, b, hi, lo);
  }
  __device__ static __forceinline__ f32x4_t mma(const V& ah, const V& al, const V& bh, const V& bl, f32x4_t c) {
    return mma3(ah, al, bh, bl, c);
  }
};
template <>
struct MmaOps<true> {
  typedef f16x8_t V;
  static constexpr int NS = 1;
  __device__ static __forceinline__ void split(const f32x4_t& a, const f32x4_t& b, V& hi, V&) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      hi[v] = (_Float16)a[v];
      hi[4 + v] = (_Float16)b[v];
    }
  }
  __device__ static __forceinline__ f32x4_t mma(const V& ah, const V&, const V& bh, const V&, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, c, 0, 0, 0);
  }
};

// Workgroups: gx tile groups x npatch patches, in an order that gives each
// XCD (workgroups go to the XCDs round robin) a contiguous range of patches of
// one tile group, so that the S rows of neighbouring patches of one sample
// (adjacent in memory) are written through the same L2.
template <bool F16>
__global__ __launch_bounds__(64 * BF_WAVES, F16 ? 4 : 1) void mlp_infer_mma_kernel(MlpInferArgs a, int gx) {
  using Ops = MmaOps<F16>;
  using V = typename Ops::V;
  constexpr int NS = Ops::NS;
  constexpr int CT = F16 ? 2 : 4;  // column tiles per pass
  const int nwg = gx * a.npatch;
  const int b = blockIdx.x;
  const int widx = (nwg % 8 == 0) ? (b % 8) * (nwg / 8) + b / 8 : b;
  const int K = widx % a.npatch, x0 = widx / a.npatch;
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  const int g = lane >> 4, col = lane & 15;
  constexpr int NT = 64 * BF_WAVES;
  __shared__ V WA[BF_OPS][NS][64];      // [operand][term][lane]
  __shared__ float2 tab[GeluLin<F16>::N];
  __shared__ float bias[3 * WD + BF_NOP];
  // the per-sample outputs of the tiles; during set-up the same memory holds
  // the patch's raw parameters
  constexpr int YS_FLOATS = BF_WAVES * 64 * (NO + 1);
  static_assert(YS_FLOATS >= MLP_NP + 4, "parameter staging must fit the output buffer");
  __shared__ __align__(16) float ysbuf[YS_FLOATS];
  float(*Ys)[64][NO + 1] = reinterpret_cast<float(*)[64][NO + 1]>(ysbuf);
  const float* Pg = a.params + (int64_t)K * MLP_NP;
  // ---- raw parameters into LDS with coalesced loads ----
  for (int i = tid; i < MLP_NP; i += NT) ysbuf[i] = Pg[i];
  __syncthreads();
  const float* P = ysbuf;
  // ---- stage the weights in the permuted A layout, split hi/lo ----
  for (int e = tid; e < BF_OPS * 64 * 8; e += NT) {
    const int j = e & 7, ln = (e >> 3) & 63, op = e >> 9;
    const int i = ln & 15, gg = ln >> 4;
    float v = 0.0f;
    if (op < BF_OPS_L2) {  // layer 1: k slot = input index
      const int nt = op, kin = 8 * gg + j;
      if (kin < MLP_KIN) v = P[MLP_OW1 + kin * WD + 16 * nt + i];
    } else {
      const int L = op < BF_OPS_L3 ? 2 : (op < BF_OPS_L4 ? 3 : 4);
      const int rel = op - (L == 2 ? BF_OPS_L2 : (L == 3 ? BF_OPS_L3 : BF_OPS_L4));
      const int nt = rel >> 1, kb = rel & 1;
      const int nin = 32 * kb + (j < 4 ? 4 * gg + j : 16 + 4 * gg + (j - 4));
      const int nout = 16 * nt + i;
      if (L == 2) v = P[MLP_OW2 + nin * WD + nout];
      else if (L == 3) v = P[MLP_OW3 + nin * WD + nout];
      else if (nout < NO) v = P[MLP_OW4 + nin * NO + nout];
    }
    V* dst[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) dst[t] = &WA[op][t][ln];
    if constexpr (NS == 2) {
      const __bf16 h = (__bf16)v;
      (*dst[0])[j] = h;
      (*dst[1])[j] = (__bf16)(v - (float)h);
    } else {
      (*dst[0])[j] = (_Float16)v;
    }
  }
  for (int i = tid; i < 3 * WD + BF_NOP; i += NT) {
    float v;
    if (i < WD) v = P[MLP_OB1 + i];
    else if (i < 2 * WD) v = P[MLP_OB2 + i - WD];
    else if (i < 3 * WD) v = P[MLP_OB3 + i - 2 * WD];
    else v = (i - 3 * WD) < NO ? P[MLP_OB4 + i - 3 * WD] : 0.0f;
    bias[i] = v;
  }
  // ---- GELU table: value and increment of Phi at each node ----
  for (int i = tid; i < GeluLin<F16>::N; i += NT) {
    const double h = 1.0 / GeluLin<F16>::SCALE, x0 = -6.0 + i * h;
    const double f0 = 0.5 * erfc(-x0 * 0.70710678118654752440);
    const double f1 = 0.5 * erfc(-(x0 + h) * 0.70710678118654752440);
    tab[i] = make_float2((float)f0, (float)(f1 - f0));
  }
  __syncthreads();
  const int lv0 = a.lv[K * MLP_KIN + 0], lv1 = a.lv[K * MLP_KIN + 1], lv2 = a.lv[K * MLP_KIN + 2],
            lv3 = a.lv[K * MLP_KIN + 3];
  const int64_t ntiles = (a.nsamples + BF_TILE - 1) / BF_TILE;
  for (int64_t tile = x0; tile < ntiles; tile += gx) {
    const int64_t wbase = tile * BF_TILE + 64 * w;  // this wavefront's 64 samples
    // CT column tiles of 16 samples go through each layer together: every A
    // operand is read from LDS once per layer and pass and used CT times
    // (BF16: one pass of four tiles; FP16: two passes of two, which keeps
    // the wavefront within the registers of four wavefronts per SIMD)
    const f32x4_t z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int hf = 0; hf < 4 / CT; ++hf) {
    V bh[CT][2], bl[CT][2];
    f32x4_t acc[CT][4];
#pragma unroll
    for (int st = 0; st < CT; ++st) {
      const int64_t s = wbase + 16 * (hf * CT + st) + col;
      f32x4_t x4 = z4;  // layer-1 B operand: x in slots 0..3 of lane group 0
      if (g == 0 && s < a.nsamples) {
        const double* xs = a.xi + s * a.nxi;
        x4[0] = lv0 >= 0 ? (float)mlp_input(a.family, xs[lv0]) : 0.0f;
        x4[1] = lv1 >= 0 ? (float)mlp_input(a.family, xs[lv1]) : 0.0f;
        x4[2] = lv2 >= 0 ? (float)mlp_input(a.family, xs[lv2]) : 0.0f;
        x4[3] = lv3 >= 0 ? (float)mlp_input(a.family, xs[lv3]) : 0.0f;
      }
      Ops::split(x4, z4, bh[st][0], bl[st][0]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const V ah = WA[BF_OPS_L1 + nt][0][lane], al = WA[BF_OPS_L1 + nt][NS - 1][lane];
      f32x4_t b4;
#pragma unroll
      for (int v = 0; v < 4; ++v) b4[v] = bias[16 * nt + 4 * g + v];
#pragma unroll
      for (int st = 0; st < CT; ++st) acc[st][nt] = Ops::mma(ah, al, bh[st][0], bl[st][0], b4);
    }
#pragma unroll
    for (int L = 0; L < 2; ++L) {
#pragma unroll
      for (int st = 0; st < CT; ++st) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[st][nt][v] = gelu_lin<F16>(tab, acc[st][nt][v]);
        Ops::split(acc[st][0], acc[st][1], bh[st][0], bl[st][0]);
        Ops::split(acc[st][2], acc[st][3], bh[st][1], bl[st][1]);
      }
      const int ob = L == 0 ? BF_OPS_L2 : BF_OPS_L3;
      const float* bs = bias + (L + 1) * WD;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4_t b4;
#pragma unroll
        for (int v = 0; v < 4; ++v) b4[v] = bs[16 * nt + 4 * g + v];
#pragma unroll
        for (int st = 0; st < CT; ++st) acc[st][nt] = b4;
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
          const V ah = WA[ob + 2 * nt + kb][0][lane], al = WA[ob + 2 * nt + kb][NS - 1][lane];
#pragma unroll
          for (int st = 0; st < CT; ++st) acc[st][nt] = Ops::mma(ah, al, bh[st][kb], bl[st][kb], acc[st][nt]);
        }
      }
    }
#pragma unroll
    for (int st = 0; st < CT; ++st) {
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[st][nt][v] = gelu_lin<F16>(tab, acc[st][nt][v]);
      Ops::split(acc[st][0], acc[st][1], bh[st][0], bl[st][0]);
      Ops::split(acc[st][2], acc[st][3], bh[st][1], bl[st][1]);
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x4_t b4;
#pragma unroll
      for (int v = 0; v < 4; ++v) b4[v] = bias[3 * WD + 16 * nt + 4 * g + v];
#pragma unroll
      for (int st = 0; st < CT; ++st) acc[st][nt] = b4;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const V ah = WA[BF_OPS_L4 + 2 * nt + kb][0][lane], al = WA[BF_OPS_L4 + 2 * nt + kb][NS - 1][lane];
#pragma unroll
        for (int st = 0; st < CT; ++st) acc[st][nt] = Ops::mma(ah, al, bh[st][kb], bl[st][kb], acc[st][nt]);
      }
    }
#pragma unroll
    for (int st = 0; st < CT; ++st)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = 16 * nt + 4 * g + v;
          if (o < NO) Ys[w][16 * (hf * CT + st) + col][o] = acc[st][nt][v];
        }
    }  // passes
    // Ys[w] is this wavefront's alone: a wavefront-level barrier orders its
    // writes before the reads of other lanes, and the wavefronts of the
    // workgroup run through their tiles independently
    wave_lds_sync();
    // ---- one sample per lane: outputs, gate, fallback list ----
    const int64_t s = wbase + lane;
    bool fb = false;
    if (s < a.nsamples) {
      const int64_t p = s * a.npatch + K;
      float yv[NO];
#pragma unroll
      for (int o = 0; o < NO; ++o) yv[o] = Ys[w][lane][o];
      if (a.Y) {
        for (int o = 0; o < NO; ++o) a.Y[p * NO + o] = yv[o];
      }
      if (a.S) gate_and_store(a, K, s, yv, a.S + p * 10, a.status ? a.status + p : nullptr, &fb);
    }
    if (a.S) {
      const unsigned long long mask = __ballot(fb);
      if (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd((unsigned long long*)a.count, (unsigned long long)__popcll(mask));
        base = __shfl(base, leader);
        if (fb) a.list[base + __popcll(mask & ((1ull << lane) - 1ull))] = s * a.npatch + K;
      }
    }
    wave_lds_sync();  // the reads of Ys[w] before the next tile's writes
  }  // tiles
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Plain solve of the listed pairs (m = 8), coefficients regenerated from xi,
// one lane per pair.  The statistics are combined over the wavefront before
// one atomic per counter.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

__global__ __launch_bounds__(64) void mlp_fallback_kernel(MlpInferArgs a) {
  __shared__ double blk[64][64];  // one 8 x 8 coefficient block per lane
  // each lane's sample's xi, staged in LDS (column per lane) when the family
  // has at most XL of them: the bump sums over the 64 elements then read
  // them from LDS instead of issuing a dependent global load per candidate
  // bump; 40 KB per workgroup keeps four workgroups (one per SIMD) per CU
  constexpr int XL = 16;
  __shared__ double xl[XL][64];
  const int lane = threadIdx.x;
  const unsigned long long count = *a.count;
  const double h = 1.0 / (a.ncx * 8);
  const BumpParams bp{a.bump_g, a.bump_rho, a.bump_eps, a.bump_base, a.bump_amp, a.bump_beta};
  // wavefront-uniform loop: every lane takes part in the statistics
  for (unsigned long long base = (unsigned long long)blockIdx.x * 64; base < count;
       base += (unsigned long long)gridDim.x * 64) {
    const unsigned long long idx = base + lane;
    bool rejected = false, audited = false;
    double rel = 0.0;
    if (idx < count) {
      const int64_t p = a.list[idx];
      const int64_t s = p / a.npatch;
      const int K = (int)(p - s * a.npatch);
      const int kx = K % a.ncx, ky = K / a.ncx;
      // the coefficient of each fine element, as the coefficient kernel forms
      // it (same operations, so the same bits); the oscillation's sines are
      // shared by the element rows and columns of the patch
      double sxv[8], syv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double xq = (kx * 8 + q + 0.5) * h, yq = (ky * 8 + q + 0.5) * h;
        sxv[q] = sin(2.0 * M_PI * xq / bp.eps);
        syv[q] = sin(2.0 * M_PI * yq / bp.eps);
      }
      const double* xs = a.xi + s * a.nxi;
      const int nb = bp.g * bp.g;
      auto regen = [&](auto xsc, const double* src) {
        constexpr int XS = decltype(xsc)::value;
#pragma unroll
        for (int ey = 0; ey < 8; ++ey)
#pragma unroll
          for (int ex = 0; ex < 8; ++ex) {
            const double x = (kx * 8 + ex + 0.5) * h, y = (ky * 8 + ey + 0.5) * h;
            const double field = bump_field<XS>(x, y, src, bp);
            const double osc = bp.base + bp.amp * sxv[ex] * syv[ey];
            blk[lane][8 * ey + ex] = osc * exp(bp.beta * field);
          }
      };
      if (nb <= XL) {
        for (int j = 0; j < nb; ++j) xl[j][lane] = xs[j];
        regen(std::integral_constant<int, 64>{}, &xl[0][lane]);
      } else {
        regen(std::integral_constant<int, 1>{}, xs);
      }
      double Sp[10];
      int32_t st = 0;
      small_cell_solve<8, double>(&blk[lane][0], 8, Sp, &st);
      double* So = a.S + p * 10;
      double err = 0.0, sc = 0.0;
      for (int q = 0; q < 10; ++q) {
        err = fmax(err, fabs(So[q] - Sp[q]));
        sc = fmax(sc, fabs(Sp[q]));
        So[q] = Sp[q];
      }
      rel = sc > 0 ? err / sc : 0.0;
      audited = a.status && a.status[p] == MLP_ST_AUDIT;
      rejected = !audited;
      if (a.status) a.status[p] = st != STOMSFEM_OK ? st : (audited ? MLP_ST_AUDIT : MLP_ST_FALLBACK);
    }
    if (a.stats) {
      const unsigned long long nrej = __popcll(__ballot(rejected)), naud = __popcll(__ballot(audited));
      const unsigned long long mrej = wave_max_u64(rejected ? (unsigned long long)__double_as_longlong(rel) : 0ull);
      const unsigned long long maud = wave_max_u64(audited ? (unsigned long long)__double_as_longlong(rel) : 0ull);
      if (lane == 0) {
        if (nrej) {
          atomicAdd(&a.stats[0], nrej);
          atomicMax(&a.stats[2], mrej);
        }
        if (naud) {
          atomicAdd(&a.stats[1], naud);
          atomicMax(&a.stats[3], maud);
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void mlp_fallback_finish_kernel(const int64_t* __restrict__ list, int64_t count,
                                                                  const double* __restrict__ Sc,
                                                                  const int32_t* __restrict__ stc, double* S,
                                                                  int32_t* status, unsigned long long* stats) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const int64_t p = list[i];
  double* So = S + p * 10;
  double err = 0.0, sc = 0.0;
  for (int q = 0; q < 10; ++q) {
    const double v = Sc[i * 10 + q];
    err = fmax(err, fabs(So[q] - v));
    sc = fmax(sc, fabs(v));
    So[q] = v;
  }
  const double rel = sc > 0 ? err / sc : 0.0;
  const bool audited = status && status[p] == MLP_ST_AUDIT;
  if (stats) {
    atomicAdd(&stats[audited ? 1 : 0], 1ull);
    atomicMax(&stats[audited ? 3 : 2], (unsigned long long)__double_as_longlong(rel));
  }
  if (status) status[p] = stc[i] != STOMSFEM_OK ? stc[i] : (audited ? MLP_ST_AUDIT : MLP_ST_FALLBACK);
}

hipError_t launch_mlp_fallback_finish(const int64_t* list, int64_t count, const double* Sc, const int32_t* stc,
                                      double* S, int32_t* status, unsigned long long* stats, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_fallback_finish_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, list, count,
                     Sc, stc, S, status, stats);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(const MlpInferArgs& a, int mode, hipStream_t st) {
  if (a.S) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, (unsigned long long*)a.count, 1);
  }
  if (mode == MLP_MODE_BF16 || mode == MLP_MODE_F16) {
    const int64_t ntiles = (a.nsamples + BF_TILE - 1) / BF_TILE;
    // workgroups persistent over their patch's tiles, so the per-workgroup
    // set-up (weights, GELU table) is paid once per workgroup: about one
    // workgroup per CU slot (BF16: one per CU, its LDS allows no second one;
    // FP16: two per CU)
    const int64_t slots = mode == MLP_MODE_F16 ? 512 : 256;
    int64_t gx = (slots + a.npatch - 1) / a.npatch;
    if (gx > ntiles) gx = ntiles;
    if (gx < 1) gx = 1;
    const dim3 grid((unsigned)(gx * a.npatch));
    if (mode == MLP_MODE_F16)
      hipLaunchKernelGGL(mlp_infer_mma_kernel<true>, grid, dim3(64 * BF_WAVES), 0, st, a, (int)gx);
    else
      hipLaunchKernelGGL(mlp_infer_mma_kernel<false>, grid, dim3(64 * BF_WAVES), 0, st, a, (int)gx);
  } else {
    const dim3 grid((unsigned)((a.nsamples + 63) / 64), (unsigned)a.npatch);
    hipLaunchKernelGGL(mlp_infer_f32_kernel, grid, dim3(64), 0, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.S || a.m != 8 || a.family != MLP_FAMILY_BUMPS) return e;
  // the listed count is known only on the device: enough wavefronts for
  // about 3% of the pairs in one pass, looping beyond that
  int64_t blocks = (a.nsamples * a.npatch / 32 + 63) / 64;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(mlp_fallback_kernel, dim3((unsigned)blocks), dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace stomsfem
