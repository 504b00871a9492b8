// Fine-grid FEM solves for large fine meshes (the u_h of the two-level Monte
// Carlo estimator, Sec. 4.1.1): the global Q1 system K u = b on the
// nfine x nfine mesh of [0,1]^2 with a piecewise-constant coefficient a_e,
// f = 1 (b = h^2 at every interior node) and zero Dirichlet data, solved by
// conjugate gradients preconditioned with one geometric multigrid V-cycle,
// for a batch of samples at once.
//
// Multigrid: level l + 1 halves the element count per side while it is even
// and at least 8; its coefficient is the mean of the four children and its
// operator the Q1 stiffness of that coefficient (rediscretisation).
// Transfers: bilinear interpolation P of the Q1 nodal values and its
// transpose for residuals.  Smoother: damped Jacobi (weight 0.8), two sweeps
// before and two after the coarse correction, the first from zero; the
// coarsest level takes thirty sweeps from zero.  The V-cycle is a fixed
// symmetric positive-definite linear operator (Jacobi is self-adjoint, the
// pre- and post-smoothers are the same, restriction is P^T), as CG needs.
//
// Layout per level and sample: nodes (n+1) x (n+1) with the boundary nodes
// kept at zero (every kernel writes interior nodes only), elements n x n;
// sample s of a chunk at offset s (n+1)^2 (nodes) or s n^2 (elements).
// Every kernel takes grid (node blocks, samples).  Dot products: one partial
// per block, summed per sample in block order (a fixed summation order).
#include "common.h"

namespace stomsfem {

constexpr int FMG_TB = 256;          // threads per block
constexpr int FMG_NPB = 4;           // nodes per thread in the dot-product kernels
constexpr double FMG_OMEGA = 0.8;    // Jacobi weight
constexpr int FMG_COARSE_SWEEPS = 30;

struct FmgLevel {
  int n;            // elements per side
  const double* a;  // [N][n][n]
  double* x;        // [N][(n+1)^2]: the level's solution (level 0: z = M r)
  double* t;        // Jacobi scratch
  double* b;        // right-hand side (level 0: the CG residual)
  double* r;        // residual
};

__device__ __forceinline__ double apply9(const double* __restrict__ a, int n, int ix, int iy,
                                         const double* __restrict__ x, double* diag) {
  const int W = n + 1;
  const double aSW = a[(iy - 1) * n + ix - 1], aSE = a[(iy - 1) * n + ix];
  const double aNW = a[iy * n + ix - 1], aNE = a[iy * n + ix];
  const double kc = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
  const double* xc = x + iy * W + ix;
  double v = kc * xc[0];
  v -= ((aSW + aNW) * xc[-1] + (aSE + aNE) * xc[1] + (aSW + aSE) * xc[-W] + (aNW + aNE) * xc[W]) * (1.0 / 6.0);
  v -= (aSW * xc[-W - 1] + aSE * xc[-W + 1] + aNW * xc[W - 1] + aNE * xc[W + 1]) * (1.0 / 3.0);
  *diag = kc;
  return v;
}

// mode 0: out = w D^{-1} b (Jacobi sweep from zero); 1: out = x + w D^{-1}(b - A x);
// 2: out = b - A x
template <int MODE>
__global__ __launch_bounds__(FMG_TB) void fmg_sweep_kernel(FmgLevel L, const double* __restrict__ x,
                                                           double* __restrict__ out) {
  const int n = L.n, W = n + 1;
  const int node = blockIdx.x * FMG_TB + threadIdx.x;
  if (node >= W * W) return;
  const int iy = node / W, ix = node - iy * W;
  if (ix == 0 || iy == 0 || ix == n || iy == n) return;
  const int64_t s = blockIdx.y;
  const double* a = L.a + s * n * n;
  const int64_t off = s * W * W;
  if (MODE == 0) {
    const double aSW = a[(iy - 1) * n + ix - 1], aSE = a[(iy - 1) * n + ix];
    const double aNW = a[iy * n + ix - 1], aNE = a[iy * n + ix];
    const double kc = (2.0 / 3.0) * ((aSW + aSE) + (aNW + aNE));
    out[off + node] = FMG_OMEGA * L.b[off + node] / kc;
  } else {
    double d;
    const double ax = apply9(a, n, ix, iy, x + off, &d);
    const double res = L.b[off + node] - ax;
    out[off + node] = MODE == 1 ? x[off + node] + FMG_OMEGA * res / d : res;
  }
}

// coarse element coefficient = mean of its four children
__global__ __launch_bounds__(FMG_TB) void fmg_coef_kernel(const double* __restrict__ af, int nf,
                                                          double* __restrict__ ac) {
  const int nc = nf / 2;
  const int e = blockIdx.x * FMG_TB + threadIdx.x;
  if (e >= nc * nc) return;
  const int64_t s = blockIdx.y;
  const int ey = e / nc, ex = e - ey * nc;
  const double* f = af + s * nf * nf + (2 * ey) * nf + 2 * ex;
  ac[s * nc * nc + e] = 0.25 * ((f[0] + f[1]) + (f[nf] + f[nf + 1]));
}

// coarse right-hand side = P^T r (full weighting)
__global__ __launch_bounds__(FMG_TB) void fmg_restrict_kernel(const double* __restrict__ rf, int nf,
                                                              double* __restrict__ bc) {
  const int nc = nf / 2, Wc = nc + 1, Wf = nf + 1;
  const int node = blockIdx.x * FMG_TB + threadIdx.x;
  if (node >= Wc * Wc) return;
  const int iy = node / Wc, ix = node - iy * Wc;
  if (ix == 0 || iy == 0 || ix == nc || iy == nc) return;
  const int64_t s = blockIdx.y;
  const double* r = rf + s * Wf * Wf + (2 * iy) * Wf + 2 * ix;
  const double v = r[0] + 0.5 * ((r[-1] + r[1]) + (r[-Wf] + r[Wf])) +
                   0.25 * ((r[-Wf - 1] + r[-Wf + 1]) + (r[Wf - 1] + r[Wf + 1]));
  bc[s * Wc * Wc + node] = v;
}

// x_f += P x_c (bilinear interpolation of the coarse nodal values)
__global__ __launch_bounds__(FMG_TB) void fmg_prolong_kernel(const double* __restrict__ xc, int nf,
                                                             double* __restrict__ xf) {
  const int nc = nf / 2, Wc = nc + 1, Wf = nf + 1;
  const int node = blockIdx.x * FMG_TB + threadIdx.x;
  if (node >= Wf * Wf) return;
  const int iy = node / Wf, ix = node - iy * Wf;
  if (ix == 0 || iy == 0 || ix == nf || iy == nf) return;
  const int64_t s = blockIdx.y;
  const double* c = xc + s * Wc * Wc;
  const int cx = ix >> 1, cy = iy >> 1;
  double v;
  if (!(ix & 1) && !(iy & 1)) {
    v = c[cy * Wc + cx];
  } else if (!(iy & 1)) {
    v = 0.5 * (c[cy * Wc + cx] + c[cy * Wc + cx + 1]);
  } else if (!(ix & 1)) {
    v = 0.5 * (c[cy * Wc + cx] + c[(cy + 1) * Wc + cx]);
  } else {
    v = 0.25 * ((c[cy * Wc + cx] + c[cy * Wc + cx + 1]) + (c[(cy + 1) * Wc + cx] + c[(cy + 1) * Wc + cx + 1]));
  }
  xf[s * Wf * Wf + node] += v;
}

// ---- conjugate gradients on level 0 ----
struct FmgCg {
  int n;
  int64_t nsamples;
  const double* a;
  double *x, *r, *z, *p, *q;
  double* part;      // [N][nblk] partial sums
  int nblk;
  double *rz, *pq, *rr, *bb, *alpha, *beta;  // [N]
  int32_t* active;   // [N]
  int32_t* iters;    // [N] iterations to convergence (or the cap)
  unsigned int* nactive;
  double tol2;
};

__device__ __forceinline__ void block_partial(double v, double* part) {
  __shared__ double red[FMG_TB];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = FMG_TB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *part = red[0];
}

// r = b = h^2 (interior), x = 0 (already), partial of b.b
__global__ __launch_bounds__(FMG_TB) void fmg_cg_init_kernel(FmgCg c) {
  const int n = c.n, W = n + 1;
  const int64_t s = blockIdx.y;
  const double h2 = 1.0 / ((double)n * n);
  double acc = 0.0;
  for (int k = 0; k < FMG_NPB; ++k) {
    const int node = (blockIdx.x * FMG_NPB + k) * FMG_TB + threadIdx.x;
    if (node >= W * W) break;
    const int iy = node / W, ix = node - iy * W;
    if (ix == 0 || iy == 0 || ix == n || iy == n) continue;
    c.r[s * W * W + node] = h2;
    acc += h2 * h2;
  }
  block_partial(acc, c.part + s * c.nblk + blockIdx.x);
}

// partial of u.v over the interior nodes
__global__ __launch_bounds__(FMG_TB) void fmg_dot_kernel(FmgCg c, const double* __restrict__ u,
                                                         const double* __restrict__ v) {
  const int n = c.n, W = n + 1;
  const int64_t s = blockIdx.y;
  double acc = 0.0;
  for (int k = 0; k < FMG_NPB; ++k) {
    const int node = (blockIdx.x * FMG_NPB + k) * FMG_TB + threadIdx.x;
    if (node >= W * W) break;
    acc += u[s * W * W + node] * v[s * W * W + node];  // boundary entries are zero
  }
  block_partial(acc, c.part + s * c.nblk + blockIdx.x);
}

// q = A p and the partial of p.q
__global__ __launch_bounds__(FMG_TB) void fmg_apply_dot_kernel(FmgCg c) {
  const int n = c.n, W = n + 1;
  const int64_t s = blockIdx.y;
  const double* a = c.a + s * n * n;
  double acc = 0.0;
  for (int k = 0; k < FMG_NPB; ++k) {
    const int node = (blockIdx.x * FMG_NPB + k) * FMG_TB + threadIdx.x;
    if (node >= W * W) break;
    const int iy = node / W, ix = node - iy * W;
    if (ix == 0 || iy == 0 || ix == n || iy == n) continue;
    double d;
    const double qv = apply9(a, n, ix, iy, c.p + s * W * W, &d);
    c.q[s * W * W + node] = qv;
    acc += c.p[s * W * W + node] * qv;
  }
  block_partial(acc, c.part + s * c.nblk + blockIdx.x);
}

// x += alpha p, r -= alpha q, partial of r.r
__global__ __launch_bounds__(FMG_TB) void fmg_update_kernel(FmgCg c) {
  const int n = c.n, W = n + 1;
  const int64_t s = blockIdx.y;
  const double al = c.alpha[s];
  double acc = 0.0;
  for (int k = 0; k < FMG_NPB; ++k) {
    const int node = (blockIdx.x * FMG_NPB + k) * FMG_TB + threadIdx.x;
    if (node >= W * W) break;
    const int64_t i = s * W * W + node;
    c.x[i] += al * c.p[i];
    const double rv = c.r[i] - al * c.q[i];
    c.r[i] = rv;
    acc += rv * rv;
  }
  block_partial(acc, c.part + s * c.nblk + blockIdx.x);
}

// p = z + beta p
__global__ __launch_bounds__(FMG_TB) void fmg_direction_kernel(FmgCg c) {
  const int n = c.n, W = n + 1;
  const int64_t s = blockIdx.y;
  const double be = c.beta[s];
  for (int k = 0; k < FMG_NPB; ++k) {
    const int node = (blockIdx.x * FMG_NPB + k) * FMG_TB + threadIdx.x;
    if (node >= W * W) break;
    const int64_t i = s * W * W + node;
    c.p[i] = c.z[i] + be * c.p[i];
  }
}

// per-sample scalar steps (one workgroup per sample: thread t sums the
// partials t, t + 256, ... in order, then a fixed tree; a fixed order)
//   0: bb = sum, active = 1;   1: rz = sum, beta = 0 (first direction p = z);
//   2: pq = sum, alpha = active ? rz / pq : 0;
//   3: rr = sum, active &= rr > tol^2 bb (count, iterations);
//   4: beta = active ? sum / rz : 0, rz = sum
template <int STEP>
__global__ __launch_bounds__(FMG_TB) void fmg_scalar_kernel(FmgCg c, int it) {
  const int64_t s = blockIdx.x;
  __shared__ double red[FMG_TB];
  double acc = 0.0;
  for (int k = threadIdx.x; k < c.nblk; k += FMG_TB) acc += c.part[s * c.nblk + k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = FMG_TB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double v = red[0];
  if (STEP == 0) {
    c.bb[s] = v;
    c.active[s] = 1;
    c.iters[s] = 0;
  } else if (STEP == 1) {
    c.rz[s] = v;
    c.beta[s] = 0.0;
  } else if (STEP == 2) {
    c.pq[s] = v;
    c.alpha[s] = (c.active[s] && v > 0.0) ? c.rz[s] / v : 0.0;
  } else if (STEP == 3) {
    c.rr[s] = v;
    if (c.active[s]) {
      c.iters[s] = it + 1;
      if (!(v > c.tol2 * c.bb[s])) c.active[s] = 0;
    }
    if (c.active[s]) atomicAdd(c.nactive, 1u);
  } else {
    c.beta[s] = (c.active[s] && c.rz[s] > 0.0) ? v / c.rz[s] : 0.0;
    c.rz[s] = v;
  }
}

__global__ void fmg_status_kernel(FmgCg c, int32_t* status) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < c.nsamples) status[s] = c.active[s] ? STOMSFEM_ENOCONV : STOMSFEM_OK;
}

__global__ void fmg_extract_kernel(const double* __restrict__ x, int n, int64_t nsamples, double* __restrict__ u) {
  const int64_t t = (int64_t)blockIdx.x * FMG_TB + threadIdx.x;
  const int64_t nU = (int64_t)(n - 1) * (n - 1);
  if (t >= nsamples * nU) return;
  const int64_t s = t / nU;
  const int i = (int)(t - s * nU);
  const int iy = i / (n - 1) + 1, ix = i % (n - 1) + 1;
  u[t] = x[s * (int64_t)(n + 1) * (n + 1) + iy * (n + 1) + ix];
}

// ---- host side ----
static int fmg_levels(int n) {
  int L = 1;
  while (n % 2 == 0 && n >= 8) {
    n /= 2;
    ++L;
  }
  return L;
}

int64_t fine_pcg_doubles_per_sample(int nfine) {
  const int L = fmg_levels(nfine);
  int64_t d = 0;
  int n = nfine;
  for (int l = 0; l < L; ++l) {
    const int64_t P = (int64_t)(n + 1) * (n + 1);
    d += (l == 0 ? 7 : 4) * P + (l == 0 ? 0 : (int64_t)n * n);  // level 0: x r z p q t rres; others x t b r + coef
    n /= 2;
  }
  const int64_t nblk = ((int64_t)(nfine + 1) * (nfine + 1) + FMG_TB * FMG_NPB - 1) / (FMG_TB * FMG_NPB);
  return d + nblk + 8;
}

static hipError_t fmg_vcycle(FmgLevel* lv, int nlev, int l, int64_t N, hipStream_t st) {
  const FmgLevel& L = lv[l];
  const int W = L.n + 1;
  const dim3 g((unsigned)((W * W + FMG_TB - 1) / FMG_TB), (unsigned)N), b(FMG_TB);
  const bool coarsest = l == nlev - 1;
  const int sweeps = coarsest ? FMG_COARSE_SWEEPS : 2;
  hipLaunchKernelGGL(fmg_sweep_kernel<0>, g, b, 0, st, L, (const double*)nullptr, L.x);
  for (int k = 1; k < sweeps; ++k) {
    hipLaunchKernelGGL(fmg_sweep_kernel<1>, g, b, 0, st, L, (const double*)L.x, L.t);
    std::swap(lv[l].x, lv[l].t);
  }
  if (coarsest) return hipGetLastError();
  const FmgLevel& L2 = lv[l];
  hipLaunchKernelGGL(fmg_sweep_kernel<2>, g, b, 0, st, L2, (const double*)L2.x, L2.r);
  const int Wc = lv[l + 1].n + 1;
  const dim3 gc((unsigned)((Wc * Wc + FMG_TB - 1) / FMG_TB), (unsigned)N);
  hipLaunchKernelGGL(fmg_restrict_kernel, gc, b, 0, st, (const double*)L2.r, L2.n, lv[l + 1].b);
  hipError_t e = fmg_vcycle(lv, nlev, l + 1, N, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fmg_prolong_kernel, g, b, 0, st, (const double*)lv[l + 1].x, lv[l].n, lv[l].x);
  for (int k = 0; k < 2; ++k) {
    hipLaunchKernelGGL(fmg_sweep_kernel<1>, g, b, 0, st, lv[l], (const double*)lv[l].x, lv[l].t);
    std::swap(lv[l].x, lv[l].t);
  }
  return hipGetLastError();
}

// Solves one chunk of N samples (reads the active count back every four
// iterations, so it synchronises the stream); work holds
// fine_pcg_doubles_per_sample(n) N doubles.  iters [N] receives the
// iterations each sample took, status [N] (may be NULL) OK or ENOCONV.
hipError_t launch_fine_pcg(const double* a, int n, int64_t N, double tol, int max_iter, double* u, int32_t* iters,
                           int32_t* status, double* work, hipStream_t st) {
  const int nlev = fmg_levels(n);
  const int64_t P0 = (int64_t)(n + 1) * (n + 1);
  hipError_t e = hipMemsetAsync(work, 0, sizeof(double) * fine_pcg_doubles_per_sample(n) * N, st);
  if (e != hipSuccess) return e;
  double* w = work;
  auto take = [&](int64_t cnt) {
    double* p = w;
    w += cnt;
    return p;
  };
  FmgCg c{};
  c.n = n;
  c.nsamples = N;
  c.a = a;
  c.x = take(P0 * N);
  c.r = take(P0 * N);
  c.p = take(P0 * N);
  c.q = take(P0 * N);
  FmgLevel lv[16];
  int nn = n;
  for (int l = 0; l < nlev; ++l) {
    const int64_t P = (int64_t)(nn + 1) * (nn + 1);
    lv[l].n = nn;
    if (l == 0) {
      lv[l].a = a;
      lv[l].x = take(P * N);  // z
      lv[l].t = take(P * N);
      lv[l].b = c.r;          // the CG residual
      lv[l].r = take(P * N);
    } else {
      double* ac = take((int64_t)nn * nn * N);
      const dim3 ge((unsigned)(((int64_t)nn * nn + FMG_TB - 1) / FMG_TB), (unsigned)N);
      hipLaunchKernelGGL(fmg_coef_kernel, ge, dim3(FMG_TB), 0, st, lv[l - 1].a, lv[l - 1].n, ac);
      lv[l].a = ac;
      lv[l].x = take(P * N);
      lv[l].t = take(P * N);
      lv[l].b = take(P * N);
      lv[l].r = take(P * N);
    }
    nn /= 2;
  }
  c.nblk = (int)((P0 + FMG_TB * FMG_NPB - 1) / (FMG_TB * FMG_NPB));
  c.part = take((int64_t)c.nblk * N);
  c.rz = take(N);
  c.pq = take(N);
  c.rr = take(N);
  c.bb = take(N);
  c.alpha = take(N);
  c.beta = take(N);
  c.active = (int32_t*)take((N + 1) / 2);
  c.iters = iters;
  unsigned int* nactive_dev = (unsigned int*)take(1);
  c.nactive = nactive_dev;
  c.tol2 = tol * tol;
  const dim3 gd((unsigned)c.nblk, (unsigned)N), b(FMG_TB);
  const dim3 gs((unsigned)N), bs(FMG_TB);         // scalar steps: one workgroup per sample
  const dim3 gst((unsigned)((N + 63) / 64)), bst(64);  // status: one thread per sample
  hipLaunchKernelGGL(fmg_cg_init_kernel, gd, b, 0, st, c);
  hipLaunchKernelGGL(fmg_scalar_kernel<0>, gs, bs, 0, st, c, 0);
  e = fmg_vcycle(lv, nlev, 0, N, st);
  if (e != hipSuccess) return e;
  c.z = lv[0].x;
  hipLaunchKernelGGL(fmg_dot_kernel, gd, b, 0, st, c, (const double*)c.r, (const double*)c.z);
  hipLaunchKernelGGL(fmg_scalar_kernel<1>, gs, bs, 0, st, c, 0);
  hipLaunchKernelGGL(fmg_direction_kernel, gd, b, 0, st, c);
  int it = 0;
  for (; it < max_iter; ++it) {
    hipLaunchKernelGGL(fmg_apply_dot_kernel, gd, b, 0, st, c);
    hipLaunchKernelGGL(fmg_scalar_kernel<2>, gs, bs, 0, st, c, it);
    hipLaunchKernelGGL(fmg_update_kernel, gd, b, 0, st, c);
    const bool check = (it % 4 == 3) || it == max_iter - 1;
    if (check) {
      e = hipMemsetAsync(nactive_dev, 0, sizeof(unsigned int), st);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fmg_scalar_kernel<3>, gs, bs, 0, st, c, it);
    if (check) {
      unsigned int na = 0;
      e = hipMemcpyAsync(&na, nactive_dev, sizeof(na), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      if (na == 0) {
        ++it;
        break;
      }
    }
    e = fmg_vcycle(lv, nlev, 0, N, st);
    if (e != hipSuccess) return e;
    c.z = lv[0].x;
    hipLaunchKernelGGL(fmg_dot_kernel, gd, b, 0, st, c, (const double*)c.r, (const double*)c.z);
    hipLaunchKernelGGL(fmg_scalar_kernel<4>, gs, bs, 0, st, c, it);
    hipLaunchKernelGGL(fmg_direction_kernel, gd, b, 0, st, c);
  }
  if (status) hipLaunchKernelGGL(fmg_status_kernel, gst, bst, 0, st, c, status);
  const int64_t nU = (int64_t)(n - 1) * (n - 1);
  hipLaunchKernelGGL(fmg_extract_kernel, dim3((unsigned)((N * nU + FMG_TB - 1) / FMG_TB)), b, 0, st,
                     (const double*)c.x, n, N, u);
  return hipGetLastError();
}

}  // namespace stomsfem
