// Local upscaling with an FP32 factorization and FP64 residual refinement
// (mixed-precision variant of the cell solves of Sec. 2.2, eq. MsFEB; S by
// eq. stiffness_local).  One wavefront per (coarse element, sample) pair:
//
//   1. the band of K_II (half-bandwidth m, natural order) is assembled in
//      FP64 and stored in LDS in FP32;
//   2. LDL^T of the band in FP32, in place, one pivot column at a time (the
//      lanes share the rank-1 update of the (m x m) trailing triangle);
//   3. refinement for the three data sets l = 0, 1, 2 at once: X = 0, then
//      r = f^l - K_II X in FP64 (f^l = -K_IB g^l; computed as -(K u)_I with
//      u = X inside and the bilinear corner data g^l on the boundary, FP64
//      coefficient), stop when max_l |r|_inf / |f^l|_inf <= tol, otherwise
//      X += (L D L^T)^{-1} r with FP32 triangular solves;
//   4. S_ll' = sum_e a_e u^l_e . K_ref u^l'_e in FP64 (energy form): for an
//      approximate u its error is e^l . K_II e^l', quadratic in the solution
//      error; S^3 by the partition of unity as in the other kernels.
// Optionally the refined solutions themselves are written out (the
// reduced basis takes them as snapshots where the FP64 band does not fit
// LDS), and S may then be skipped.
// Pairs that do not converge within max_iter (or meet a non-positive FP32
// pivot) are appended to a list for the FP64 path.
//
// LDS per pair: band (m-1)^2 (m+1) floats, X 3 (m-1)^2 doubles, work
// 3 (m-1)^2 floats (161 KB at m = 32, 23 KB at m = 16).
#include "mixed.h"

namespace stomsfem {

// Entry of the full local stiffness between grid nodes (px, py) and (qx, qy)
// of the (m+1) x (m+1) local grid: sum over the elements containing both of
// a_e K_ref(alpha, beta) (local node numbering counter-clockwise from the
// lower-left corner).
template <typename T>
__device__ __forceinline__ double node_entry(const T* a, int64_t lda, int m, int px, int py, int qx, int qy) {
  double v = 0.0;
  for (int ey = max(max(py, qy) - 1, 0); ey <= min(min(py, qy), m - 1); ++ey)
    for (int ex = max(max(px, qx) - 1, 0); ex <= min(min(px, qx), m - 1); ++ex) {
      const int dxp = px - ex, dyp = py - ey, dxq = qx - ex, dyq = qy - ey;
      const int al = dyp ? (dxp ? 2 : 3) : (dxp ? 1 : 0);
      const int be = dyq ? (dxq ? 2 : 3) : (dxq ? 1 : 0);
      v += ld(a, (int64_t)ey * lda + ex) * kref(al, be);
    }
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T, int MC>
__global__ __launch_bounds__(64) void upscale_mixed_kernel(MixedArgs args) {
  extern __shared__ double lds_d[];
  const UpArgs& up = args.up;
  const int m = up.m, n = m - 1, NI = n * n, W = m + 1;
  float* Lb = (float*)lds_d;                                       // [NI][W], (i, i-d) at i*W + d
  double* X = lds_d + ((size_t)NI * W + 1) / 2;                    // [3][NI]
  float* Wk = (float*)(X + 3 * NI);                                // [3][NI]
  __shared__ float colv[MC];
  __shared__ int bad;
  const int lane = threadIdx.x;
  const int Mc = up.ncx * up.ncy;
  const int64_t lda = (int64_t)up.ncx * m;
  const int64_t p = blockIdx.x;
  if (p >= up.npairs) return;
  const int64_t s = p / Mc;
  const int K = (int)(p - s * Mc);
  const T* a = (const T*)up.a + block_offset(s, K, up.ncx, up.ncy, m);

  // 1. band of K_II in FP32
  for (int idx = lane; idx < NI * W; idx += 64) {
    const int i = idx / W, d = idx - (idx / W) * W, k = i - d;
    float v = 0.0f;
    if (k >= 0) {
      const int ix = i % n, iy = i / n, kx = k % n, ky = k / n;
      if (abs(ix - kx) <= 1 && abs(iy - ky) <= 1) v = (float)node_entry(a, lda, m, ix + 1, iy + 1, kx + 1, ky + 1);
    }
    Lb[idx] = v;
  }
  for (int idx = lane; idx < 3 * NI; idx += 64) X[idx] = 0.0;
  if (lane == 0) bad = 0;
  __syncthreads();

  // 2. LDL^T, in place: after column j, Lb[j*W] = d_j and Lb[i*W + (i-j)] =
  // l_ij.  Lane entries of the trailing triangle (offsets ii >= kk from j+1)
  // are fixed across columns.
  constexpr int NQ = (MC * (MC + 1) / 2 + 63) / 64;
  int tii[NQ], tkk[NQ];
  {
    const int ntri = m * (m + 1) / 2;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int t = lane + 64 * q;
      int ii = 0;
      while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
      tii[q] = t < ntri ? ii : -1;
      tkk[q] = t - ii * (ii + 1) / 2;
    }
  }
  for (int j = 0; j < NI; ++j) {
    const float dj = Lb[j * W];
    const float inv = 1.0f / dj;
    if (lane < m) {
      const int i = j + 1 + lane;
      colv[lane] = i < NI ? Lb[i * W + (i - j)] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = j + 1 + tii[q], k = j + 1 + tkk[q];
      if (tii[q] >= 0 && i < NI) Lb[i * W + (i - k)] -= colv[tii[q]] * inv * colv[tkk[q]];
    }
    if (lane < m && j + 1 + lane < NI) {
      const int i = j + 1 + lane;
      Lb[i * W + (i - j)] = colv[lane] * inv;
    }
    if (lane == 0 && !(dj > 0.0f && dj < INFINITY)) bad = 1;
    __syncthreads();
  }

  // 3. refinement
  auto u_at = [&](int l, int px, int py) -> double {
    if (px == 0 || px == m || py == 0 || py == m) return pcorner(l, px, py, m);
    return X[l * NI + (py - 1) * n + (px - 1)];
  };
  double fnorm[3] = {0.0, 0.0, 0.0};
  bool converged = false;
  for (int it = 0; it <= args.max_iter && !bad; ++it) {
    double rmax[3] = {0.0, 0.0, 0.0};
    for (int i = lane; i < NI; i += 64) {
      // 9-point row of the full local stiffness at interior node (px, py)
      const int px = i % n + 1, py = i / n + 1;
      const double aSW = ld(a, (int64_t)(py - 1) * lda + px - 1), aSE = ld(a, (int64_t)(py - 1) * lda + px);
      const double aNW = ld(a, (int64_t)py * lda + px - 1), aNE = ld(a, (int64_t)py * lda + px);
      const double kc = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
      const double kw = -(aSW + aNW) / 6.0, ke = -(aSE + aNE) / 6.0;
      const double ks = -(aSW + aSE) / 6.0, kn = -(aNW + aNE) / 6.0;
      const double ksw = -aSW / 3.0, kse = -aSE / 3.0, knw = -aNW / 3.0, kne = -aNE / 3.0;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const double r = -(kc * u_at(l, px, py) + kw * u_at(l, px - 1, py) + ke * u_at(l, px + 1, py) +
                           ks * u_at(l, px, py - 1) + kn * u_at(l, px, py + 1) + ksw * u_at(l, px - 1, py - 1) +
                           kse * u_at(l, px + 1, py - 1) + knw * u_at(l, px - 1, py + 1) +
                           kne * u_at(l, px + 1, py + 1));
        Wk[l * NI + i] = (float)r;
        rmax[l] = fmax(rmax[l], fabs(r));
      }
    }
    double worst = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      rmax[l] = wave_max(rmax[l]);
      if (it == 0) fnorm[l] = rmax[l];
      worst = fmax(worst, fnorm[l] > 0.0 ? rmax[l] / fnorm[l] : 0.0);
    }
    if (worst <= args.tol) {
      converged = true;
      break;
    }
    if (it == args.max_iter) break;
    __syncthreads();
    // forward: unit lower L, column j of L updates rows j+1 .. j+m
    for (int j = 0; j < NI; ++j) {
      for (int t = lane; t < 3 * m; t += 64) {
        const int l = t / m, i = j + 1 + (t - l * m);
        if (i < NI) Wk[l * NI + i] -= Lb[i * W + (i - j)] * Wk[l * NI + j];
      }
      __syncthreads();
    }
    for (int idx = lane; idx < 3 * NI; idx += 64) {
      const int i = idx % NI;
      Wk[idx] /= Lb[i * W];
    }
    __syncthreads();
    // backward: L^T, row j of L updates rows j-1 .. j-m
    for (int j = NI - 1; j >= 0; --j) {
      for (int t = lane; t < 3 * m; t += 64) {
        const int l = t / m, i = j - 1 - (t - l * m);
        if (i >= 0) Wk[l * NI + i] -= Lb[j * W + (j - i)] * Wk[l * NI + j];
      }
      __syncthreads();
    }
    for (int idx = lane; idx < 3 * NI; idx += 64) X[idx] += (double)Wk[idx];
    __syncthreads();
  }
  if (bad || !converged) {
    if (lane == 0) {
      const unsigned long long slot = atomicAdd(args.count, 1ull);
      args.list[slot] = p;
    }
    return;
  }

  if (!up.S) return;
  // 4. S by the element energy sum, FP64
  double e6[6] = {0, 0, 0, 0, 0, 0};
  for (int e = lane; e < m * m; e += 64) {
    const int ex = e % m, ey = e / m;
    const double ae = ld(a, (int64_t)ey * lda + ex);
    double ul[3][4];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      ul[l][0] = u_at(l, ex, ey);
      ul[l][1] = u_at(l, ex + 1, ey);
      ul[l][2] = u_at(l, ex + 1, ey + 1);
      ul[l][3] = u_at(l, ex, ey + 1);
    }
    int q = 0;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int lp = l; lp < 3; ++lp) {
        double v = 0.0;
#pragma unroll
        for (int al = 0; al < 4; ++al)
#pragma unroll
          for (int be = 0; be < 4; ++be) v += ul[l][al] * kref(al, be) * ul[lp][be];
        e6[q++] += ae * v;
      }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) e6[q] = wave_sum(e6[q]);
  if (lane == 0) {
    const double s3[3][3] = {{e6[0], e6[1], e6[2]}, {e6[1], e6[3], e6[4]}, {e6[2], e6[4], e6[5]}};
    store_packed(up.S + p * 10, s3);
    if (up.status) up.status[p] = STOMSFEM_OK;
  }
}

// Copy the coefficient blocks of listed pairs into compact FP64 blocks
// out[i][m][m].
template <typename T>
__global__ __launch_bounds__(256) void gather_blocks_kernel(UpArgs up, const int64_t* __restrict__ list,
                                                            int64_t count, double* __restrict__ out) {
  const int64_t mm = (int64_t)up.m * up.m;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= count * mm) return;
  const int64_t i = t / mm;
  const int e = (int)(t - i * mm);
  const int Mc = up.ncx * up.ncy;
  const int64_t p = list[i];
  const int64_t s = p / Mc;
  const int K = (int)(p - s * Mc);
  const T* a = (const T*)up.a + block_offset(s, K, up.ncx, up.ncy, up.m);
  out[t] = ld(a, (int64_t)(e / up.m) * ((int64_t)up.ncx * up.m) + e % up.m);
}

size_t upscale_mixed_lds_bytes(int m) {
  const size_t NI = (size_t)(m - 1) * (m - 1), W = m + 1;
  return sizeof(double) * ((NI * W + 1) / 2) + sizeof(double) * 3 * NI + sizeof(float) * 3 * NI;
}

template <typename T, int MC>
static hipError_t launch_mixed_t(const MixedArgs& a, hipStream_t st) {
  const size_t lds = upscale_mixed_lds_bytes(a.up.m);
  hipError_t e = hipFuncSetAttribute((const void*)upscale_mixed_kernel<T, MC>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((upscale_mixed_kernel<T, MC>), dim3((unsigned)a.up.npairs), dim3(64), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_upscale_mixed(const MixedArgs& a, int a_dtype, hipStream_t st) {
  if (a.up.npairs <= 0) return hipSuccess;
  const int m = a.up.m;
  if (m < 1 || m > 32) return hipErrorInvalidValue;
  const bool f32 = a_dtype == STOMSFEM_F32;
  if (m <= 8) return f32 ? launch_mixed_t<float, 8>(a, st) : launch_mixed_t<double, 8>(a, st);
  if (m <= 16) return f32 ? launch_mixed_t<float, 16>(a, st) : launch_mixed_t<double, 16>(a, st);
  return f32 ? launch_mixed_t<float, 32>(a, st) : launch_mixed_t<double, 32>(a, st);
}

hipError_t launch_gather_blocks(const UpArgs& up, int a_dtype, const int64_t* list, int64_t count, double* out,
                                hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t n = count * up.m * up.m;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (a_dtype == STOMSFEM_F32)
    hipLaunchKernelGGL(gather_blocks_kernel<float>, grid, dim3(256), 0, st, up, list, count, out);
  else
    hipLaunchKernelGGL(gather_blocks_kernel<double>, grid, dim3(256), 0, st, up, list, count, out);
  return hipGetLastError();
}

}  // namespace stomsfem
