// The short-correlation Gaussian medium (Sec. 5.3, eqs. mediaEx2 and
// betaCov) and its local KL parametrization on the coarse elements (Sec. 2.1,
// eqs. domainpar, localKL and local_KL_truncation).
//
// gauss_field_kernel: beta(x) = sqrt(2/J) sum_j cos(w_j . x + phi_j) at the
// element centroids (the randomized spectral method: w_j = sqrt(2) (z_j1/l1,
// z_j2/l2) has the normal law whose characteristic function is the
// covariance, phi_j = 2 pi u_j), kappa = 0.1 + exp(beta).  One workgroup per
// 16 x 16 tile of one sample; the sample's J terms are staged in LDS.
//
// Local KL (host): the patch covariance exp(-dx^2/l1^2 - dy^2/l2^2) on the
// m x m centroids is the Kronecker product of two m x m matrices, so its
// eigenpairs are the products of the one-dimensional ones (cyclic Jacobi);
// the K largest products give mu_k and the modes v_k = vy (x) vx.
//
// kl_project_kernel: one wavefront per (sample, element): xi_k = v_k . beta /
// sqrt(mu_k), lanes over the element's m^2 values, partial sums combined
// through LDS in a fixed order; pairs with |xi_k| > box for some k are counted.
// kl_blocks_kernel: kappa of the first K' terms on every pair's block,
// 0.1 + exp(sum_k sqrt(mu_k) xi_k v_k), one thread per element.
#include <cmath>
#include <vector>

#include "common.h"

namespace stomsfem {

constexpr int GF_TILE = 16;
constexpr int GF_JMAX = 1024;  // spectral terms per sample
constexpr int KL_KMAX = 16;    // local KL terms

__global__ __launch_bounds__(256) void gauss_field_kernel(int64_t nsamples, int nfine, int J,
                                                          const double* __restrict__ z,
                                                          const double* __restrict__ u, double l1, double l2,
                                                          double* __restrict__ beta, double* __restrict__ kappa,
                                                          int tiles_x) {
  __shared__ double w1s[GF_JMAX], w2s[GF_JMAX], phs[GF_JMAX];
  const int64_t tiles = (int64_t)tiles_x * tiles_x;
  const int64_t nblk = nsamples * tiles;
  const double h = 1.0 / nfine, amp = sqrt(2.0 / J);
  const int lane = threadIdx.x;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int64_t s = b / tiles;
    const int tt = (int)(b - s * tiles);
    const int tx = tt % tiles_x, ty = tt / tiles_x;
    __syncthreads();  // the previous tile's readers are done
    for (int j = lane; j < J; j += 256) {
      w1s[j] = sqrt(2.0) * z[(s * J + j) * 2] / l1;
      w2s[j] = sqrt(2.0) * z[(s * J + j) * 2 + 1] / l2;
      phs[j] = 2.0 * M_PI * u[s * J + j];
    }
    __syncthreads();
    const int ix = tx * GF_TILE + (lane % GF_TILE), iy = ty * GF_TILE + lane / GF_TILE;
    if (ix < nfine && iy < nfine) {
      const double x = (ix + 0.5) * h, y = (iy + 0.5) * h;
      double acc = 0.0;
      for (int j = 0; j < J; ++j) acc += cos(w1s[j] * x + w2s[j] * y + phs[j]);
      const double bv = amp * acc;
      const int64_t o = (s * nfine + iy) * (int64_t)nfine + ix;
      if (beta) beta[o] = bv;
      kappa[o] = 0.1 + exp(bv);
    }
  }
}

hipError_t launch_gauss_field(int64_t nsamples, int nfine, int J, const double* z, const double* u, double l1,
                              double l2, double* beta, double* kappa, hipStream_t st) {
  const int tiles_x = (nfine + GF_TILE - 1) / GF_TILE;
  int64_t blocks = nsamples * (int64_t)tiles_x * tiles_x;
  if (blocks == 0) return hipSuccess;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  hipLaunchKernelGGL(gauss_field_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nsamples, nfine, J, z, u, l1, l2,
                     beta, kappa, tiles_x);
  return hipGetLastError();
}

// symmetric eigenpairs of an n x n matrix by cyclic Jacobi rotations:
// eigenvalues in d, eigenvectors in the columns of V (row-major)
static void jacobi_eig(int n, std::vector<double> A, std::vector<double>& d, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        if (i != j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - sn * akq;
          A[(size_t)k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - sn * aqk;
          A[(size_t)q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
  d.resize(n);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
}

void local_kl_modes(int m, double h, double l1, double l2, int K, double* mu, double* modes, double* captured) {
  std::vector<double> Cx((size_t)m * m), Cy((size_t)m * m), dx, dy, Vx, Vy;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const double d = (i - j) * h;
      Cx[(size_t)i * m + j] = std::exp(-d * d / (l1 * l1));
      Cy[(size_t)i * m + j] = std::exp(-d * d / (l2 * l2));
    }
  jacobi_eig(m, Cx, dx, Vx);
  jacobi_eig(m, Cy, dy, Vy);
  // all m^2 products, the K largest (ties: lower (y, x) index first)
  std::vector<int> order((size_t)m * m);
  for (int i = 0; i < m * m; ++i) order[i] = i;
  auto val = [&](int i) { return dy[i / m] * dx[i % m]; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return val(a) > val(b); });
  double total = 0.0, kept = 0.0;
  for (int i = 0; i < m; ++i) total += dx[i];
  double ty = 0.0;
  for (int i = 0; i < m; ++i) ty += dy[i];
  total *= ty;
  for (int k = 0; k < K; ++k) {
    const int a = order[k], iy = a / m, ixm = a % m;
    mu[k] = val(a);
    kept += mu[k];
    for (int py = 0; py < m; ++py)
      for (int px = 0; px < m; ++px)
        modes[((size_t)k * m + py) * m + px] = Vy[(size_t)py * m + iy] * Vx[(size_t)px * m + ixm];
  }
  if (captured) *captured = kept / total;
}

__global__ __launch_bounds__(64) void kl_project_kernel(int64_t npairs, int nc, int m, int K,
                                                        const double* __restrict__ beta,
                                                        const double* __restrict__ mu,
                                                        const double* __restrict__ modes, double box,
                                                        double* __restrict__ xi, int32_t* __restrict__ outside,
                                                        unsigned long long* count) {
  __shared__ double part[KL_KMAX][64];
  const int lane = threadIdx.x;
  const int64_t p = blockIdx.x;
  const int64_t M = (int64_t)nc * nc, s = p / M;
  const int K0 = (int)(p - s * M), kx = K0 % nc, ky = K0 / nc;
  const int64_t nf = (int64_t)nc * m;
  const double* B = beta + s * nf * nf + (int64_t)ky * m * nf + (int64_t)kx * m;
  double acc[KL_KMAX];
#pragma unroll
  for (int k = 0; k < KL_KMAX; ++k) acc[k] = 0.0;
  for (int e = lane; e < m * m; e += 64) {
    const double b = B[(int64_t)(e / m) * nf + (e % m)];
#pragma unroll
    for (int k = 0; k < KL_KMAX; ++k)
      if (k < K) acc[k] += b * modes[(int64_t)k * m * m + e];
  }
#pragma unroll
  for (int k = 0; k < KL_KMAX; ++k)
    if (k < K) part[k][lane] = acc[k];
  __syncthreads();
  if (lane < K) {
    double t = 0.0;
    for (int l = 0; l < 64; ++l) t += part[lane][l];
    const double x = t / sqrt(mu[lane]);
    xi[p * K + lane] = x;
    part[lane][0] = x;
  }
  __syncthreads();
  if (lane == 0) {
    bool out = false;
    for (int k = 0; k < K; ++k) out = out || !(fabs(part[k][0]) <= box);
    if (outside) outside[p] = out ? 1 : 0;
    if (out && count) atomicAdd(count, 1ull);
  }
}

hipError_t launch_kl_project(int64_t npairs, int nc, int m, int K, const double* beta, const double* mu,
                             const double* modes, double box, double* xi, int32_t* outside,
                             unsigned long long* count, hipStream_t st) {
  if (npairs == 0) return hipSuccess;
  if (npairs > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kl_project_kernel, dim3((unsigned)npairs), dim3(64), 0, st, npairs, nc, m, K, beta, mu, modes,
                     box, xi, outside, count);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void kl_blocks_kernel(int64_t npairs, int m, int Kuse, int K,
                                                        const double* __restrict__ xi,
                                                        const double* __restrict__ mu,
                                                        const double* __restrict__ modes,
                                                        double* __restrict__ blocks) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t mm = (int64_t)m * m;
  if (t >= npairs * mm) return;
  const int64_t p = t / mm;
  const int e = (int)(t - p * mm);
  double b = 0.0;
  for (int k = 0; k < Kuse; ++k) b += sqrt(mu[k]) * xi[p * K + k] * modes[k * mm + e];
  blocks[t] = 0.1 + exp(b);
}

hipError_t launch_kl_blocks(int64_t npairs, int m, int Kuse, int K, const double* xi, const double* mu,
                            const double* modes, double* blocks, hipStream_t st) {
  const int64_t n = npairs * (int64_t)m * m;
  if (n == 0) return hipSuccess;
  const int64_t nb = (n + 255) / 256;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kl_blocks_kernel, dim3((unsigned)nb), dim3(256), 0, st, npairs, m, Kuse, K, xi, mu, modes,
                     blocks);
  return hipGetLastError();
}

}  // namespace stomsfem
