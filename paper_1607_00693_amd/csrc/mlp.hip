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
//   mlp_infer_bf16_kernel    BF16 MFMA (v_mfma_f32_16x16x16bf16_1k, FP32
//                            accumulation, three-term bf16 splitting of
//                            weights and activations, FP32 bias + GELU)
//                            inference, then the gate per pair;
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
    d.X[t * MLP_KIN + c] = j >= 0 ? (float)d.xi[s * d.nxi + j] : 0.0f;
  }
  const double* S = d.S + (s * d.npatch + K) * 10;
  for (int q = 0; q < 10; ++q) d.T[t * 10 + q] = (float)((S[q] - d.mu[K * 10 + q]) / d.sd[K * 10 + q]);
}

// Per-patch, per-entry mean and standard deviation (FP64, fixed order).
__global__ void mlp_stats_kernel(MlpDataArgs d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.npatch * 10) return;
  const int K = t / 10, q = t % 10;
  double m = 0.0;
  for (int64_t s = 0; s < d.ntrain; ++s) m += d.S[(s * d.npatch + K) * 10 + q];
  m /= (double)d.ntrain;
  double v = 0.0;
  for (int64_t s = 0; s < d.ntrain; ++s) {
    const double e = d.S[(s * d.npatch + K) * 10 + q] - m;
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
// The gate of one pair from its 20 raw outputs y (heads A and B): writes the
// stored S (P S P if accepted, else the head mean), the residual and the
// uncertainty, and returns acceptance.  A pair is accepted only if all 20
// de-standardised values are finite, max|S| > 0, both signals are <= tau and
// every local variable is inside the box; with a non-finite value the two
// signals are NaN (comparisons are written so that NaN never passes).
__device__ __forceinline__ bool gate_pair(const double* __restrict__ mu, const double* __restrict__ sd,
                                          const float* y, bool inbox, double tau, double* Sout, double* resid_out,
                                          double* unc_out) {
  double SA[10], SB[10], S[10];
  double scale = 0.0, unc = 0.0;
  bool finite = true;
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    SA[q] = mu[q] + sd[q] * (double)y[q];
    SB[q] = mu[q] + sd[q] * (double)y[10 + q];
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
    if (j >= 0 && !(fabs(a.xi[s * a.nxi + j]) <= a.box)) inbox = false;
  }
  return inbox;
}

__device__ __forceinline__ void gate_and_store(const MlpInferArgs& a, int K, int64_t s, const float* y, double* Sout,
                                               int32_t* st, bool* fallback) {
  const int64_t p = s * a.npatch + K;
  double resid, unc;
  const bool ok = gate_pair(a.mu + K * 10, a.sd + K * 10, y, local_vars_in_box(a, K, s), a.tau, Sout, &resid, &unc);
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
  const bool ok =
      gate_pair(a.mu + K * 10, a.sd + K * 10, y, local_vars_in_box(a, K, s), a.tau, a.S + p * 10, &resid, &unc);
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
    x[c] = j >= 0 ? (float)a.xi[s * a.nxi + j] : 0.0f;
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

// BF16 MFMA inference.  Workgroup = 4 wavefronts x 16 samples of one patch.
// Every FP32 weight w and activation h is carried as two bf16 numbers,
// w = w_hi + w_lo, h = h_hi + h_lo (w_hi = bf16(w), w_lo = bf16(w - w_hi)), and
// each product is formed as h_hi w_hi + h_hi w_lo + h_lo w_hi on the matrix
// cores with FP32 accumulation (the h_lo w_lo term is below FP32 rounding).
// Weights are stored transposed (n-major) so that each lane's four
// consecutive k are adjacent in LDS.
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

constexpr int BF_KIN = 16;  // layer-1 K padded to one MFMA K step
constexpr int BF_NO = 32;   // 20 outputs padded to two N tiles
constexpr int BF_LD = WD + 4;

constexpr int BF_WAVES = 8;               // wavefronts per workgroup
constexpr int BF_TILE = 16 * BF_WAVES;     // samples per tile

__global__ __launch_bounds__(64 * BF_WAVES) void mlp_infer_bf16_kernel(MlpInferArgs a) {
  using s4 = __attribute__((__vector_size__(4 * sizeof(short)))) short;
  using f4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
  const int K = blockIdx.y;
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  constexpr int NT = 64 * BF_WAVES;
  // [2] = hi, lo
  __shared__ uint16_t W1t[2][WD][BF_KIN], W2t[2][WD][BF_LD], W3t[2][WD][BF_LD], W4t[2][BF_NO][BF_LD];
  __shared__ float bias[3 * WD + BF_NO];
  __shared__ uint16_t Hs[BF_WAVES][2][2][16][BF_LD];  // wave, ping-pong buffer, hi/lo, row, k
  __shared__ float Ys[BF_WAVES][16][BF_NO + 1];
  const float* P = a.params + (int64_t)K * MLP_NP;
  auto split = [](float v, uint16_t& hi, uint16_t& lo) {
    hi = to_bf16(v);
    lo = to_bf16(v - from_bf16(hi));
  };
  for (int i = tid; i < WD * BF_KIN; i += NT) {
    const int nn = i / BF_KIN, k = i % BF_KIN;
    split(k < MLP_KIN ? P[MLP_OW1 + k * WD + nn] : 0.0f, W1t[0][nn][k], W1t[1][nn][k]);
  }
  for (int i = tid; i < WD * WD; i += NT) {
    const int nn = i / WD, k = i % WD;
    split(P[MLP_OW2 + k * WD + nn], W2t[0][nn][k], W2t[1][nn][k]);
    split(P[MLP_OW3 + k * WD + nn], W3t[0][nn][k], W3t[1][nn][k]);
  }
  for (int i = tid; i < BF_NO * WD; i += NT) {
    const int nn = i / WD, k = i % WD;
    split(nn < NO ? P[MLP_OW4 + k * NO + nn] : 0.0f, W4t[0][nn][k], W4t[1][nn][k]);
  }
  for (int i = tid; i < 3 * WD + BF_NO; i += NT) {
    float v;
    if (i < WD) v = P[MLP_OB1 + i];
    else if (i < 2 * WD) v = P[MLP_OB2 + i - WD];
    else if (i < 3 * WD) v = P[MLP_OB3 + i - 2 * WD];
    else v = (i - 3 * WD) < NO ? P[MLP_OB4 + i - 3 * WD] : 0.0f;
    bias[i] = v;
  }
  const int64_t ntiles = (a.nsamples + BF_TILE - 1) / BF_TILE;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
  __syncthreads();
  // inputs of this wavefront's 16 samples (row = sample, k < 4 used)
  const int64_t sbase = tile * BF_TILE + 16 * w;
  for (int i = lane; i < 16 * BF_KIN; i += 64) {
    const int r = i / BF_KIN, k = i % BF_KIN;
    const int64_t s = sbase + r;
    float v = 0.0f;
    if (k < MLP_KIN && s < a.nsamples) {
      const int j = a.lv[K * MLP_KIN + k];
      v = j >= 0 ? (float)a.xi[s * a.nxi + j] : 0.0f;
    }
    split(v, Hs[w][0][0][r][k], Hs[w][0][1][r][k]);
  }
  __syncthreads();
  const int row = lane & 15, kq = lane >> 4;  // A: row, k group; B: column, k group
  auto loadA = [&](int buf, int part, int k0) {
    s4 v;
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = (short)Hs[w][buf][part][row][k0 + 4 * kq + t];
    return v;
  };
  auto store_act = [&](int buf, int ntile, const f4& c, int boff) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * kq + v, col = 16 * ntile + (lane & 15);
      split(gelu_f(c[v] + bias[boff + col]), Hs[w][buf][0][r][col], Hs[w][buf][1][r][col]);
    }
  };
  auto mma3 = [](const s4& ah, const s4& al, const s4& bh, const s4& bl, f4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
  };
  // layer 1: [16 x 16] x [16 x 64]
  {
    const s4 ah = loadA(0, 0, 0), al = loadA(0, 1, 0);
    f4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      s4 bh, bl;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        bh[t] = (short)W1t[0][16 * nt + row][4 * kq + t];
        bl[t] = (short)W1t[1][16 * nt + row][4 * kq + t];
      }
      acc[nt] = mma3(ah, al, bh, bl, f4{0.f, 0.f, 0.f, 0.f});
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) store_act(1, nt, acc[nt], 0);
  }
  __syncthreads();
  // layers 2 and 3: [16 x 64] x [64 x 64]
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const int inb = layer == 0 ? 1 : 0, outb = layer == 0 ? 0 : 1;  // ping-pong activation buffers
    f4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const s4 ah = loadA(inb, 0, 16 * kk), al = loadA(inb, 1, 16 * kk);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        s4 bh, bl;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int nn = 16 * nt + row, k = 16 * kk + 4 * kq + t;
          bh[t] = (short)(layer == 0 ? W2t[0][nn][k] : W3t[0][nn][k]);
          bl[t] = (short)(layer == 0 ? W2t[1][nn][k] : W3t[1][nn][k]);
        }
        acc[nt] = mma3(ah, al, bh, bl, acc[nt]);
      }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) store_act(outb, nt, acc[nt], (layer + 1) * WD);
    __syncthreads();
  }
  // layer 4: [16 x 64] x [64 x 32], FP32 output + bias
  {
    f4 acc[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const s4 ah = loadA(1, 0, 16 * kk), al = loadA(1, 1, 16 * kk);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        s4 bh, bl;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          bh[t] = (short)W4t[0][16 * nt + row][16 * kk + 4 * kq + t];
          bl[t] = (short)W4t[1][16 * nt + row][16 * kk + 4 * kq + t];
        }
        acc[nt] = mma3(ah, al, bh, bl, acc[nt]);
      }
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * kq + v, col = 16 * nt + (lane & 15);
        Ys[w][r][col] = acc[nt][v] + bias[3 * WD + col];
      }
  }
  __syncthreads();
  if (lane < 16) {
    const int64_t s = sbase + lane;
    if (s < a.nsamples) {
      const int64_t p = s * a.npatch + K;
      float y[NO];
#pragma unroll
      for (int o = 0; o < NO; ++o) y[o] = Ys[w][lane][o];
      if (a.Y) {
        for (int o = 0; o < NO; ++o) a.Y[p * NO + o] = y[o];
      }
      if (a.S) {
        bool fb;
        gate_and_store(a, K, s, y, a.S + p * 10, a.status ? a.status + p : nullptr, &fb);
        if (fb) push_fallback(a, p);
      }
    }
  }
  }  // tiles
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Plain solve of the listed pairs (m = 8), coefficients regenerated from xi.
__global__ __launch_bounds__(64) void mlp_fallback_kernel(MlpInferArgs a) {
  __shared__ double blk[64][64];
  const int lane = threadIdx.x;
  const unsigned long long count = *a.count;
  const double h = 1.0 / (a.ncx * 8);
  const BumpParams bp{a.bump_g, a.bump_rho, a.bump_eps, a.bump_base, a.bump_amp, a.bump_beta};
  for (unsigned long long idx = (unsigned long long)blockIdx.x * 64 + lane; idx < count;
       idx += (unsigned long long)gridDim.x * 64) {
    const int64_t p = a.list[idx];
    const int64_t s = p / a.npatch;
    const int K = (int)(p - s * a.npatch);
    const int kx = K % a.ncx, ky = K / a.ncx;
    for (int e = 0; e < 64; ++e) {
      const int ex = e % 8, ey = e / 8;
      blk[lane][e] = bump_coef((kx * 8 + ex + 0.5) * h, (ky * 8 + ey + 0.5) * h, a.xi + s * a.nxi, bp);
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
    const double rel = sc > 0 ? err / sc : 0.0;
    const bool audited = a.status && a.status[p] == MLP_ST_AUDIT;
    if (a.stats) {
      atomicAdd(&a.stats[audited ? 1 : 0], 1ull);
      atomicMax(&a.stats[audited ? 3 : 2], (unsigned long long)__double_as_longlong(rel));
    }
    if (a.status) a.status[p] = st != STOMSFEM_OK ? st : (audited ? MLP_ST_AUDIT : MLP_ST_FALLBACK);
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

hipError_t launch_mlp_infer(const MlpInferArgs& a, bool bf16, hipStream_t st) {
  if (a.S) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, (unsigned long long*)a.count, 1);
  }
  if (bf16) {
    const int64_t ntiles = (a.nsamples + BF_TILE - 1) / BF_TILE;
    int64_t gx = (1024 + a.npatch - 1) / a.npatch;  // about four workgroups per CU in total
    if (gx > ntiles) gx = ntiles;
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(mlp_infer_bf16_kernel, dim3((unsigned)gx, (unsigned)a.npatch), dim3(64 * BF_WAVES), 0, st, a);
  } else {
    const dim3 grid((unsigned)((a.nsamples + 63) / 64), (unsigned)a.npatch);
    hipLaunchKernelGGL(mlp_infer_f32_kernel, grid, dim3(64), 0, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.S || a.m != 8) return e;
  int64_t blocks = (a.nsamples * a.npatch + 63) / 64;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(mlp_fallback_kernel, dim3((unsigned)blocks), dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace stomsfem
