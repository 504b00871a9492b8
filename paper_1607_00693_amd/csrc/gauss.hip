// The short-correlation Gaussian medium (Sec. 5.3, eqs. mediaEx2 and
// betaCov) and its local KL parametrization on the coarse elements (Sec. 2.1,
// eqs. domainpar, localKL and local_KL_truncation).
//
// gauss_field_kernel: beta(x) = sqrt(2/J) sum_j cos(w_j . x + phi_j) at the
// element centroids (the randomized spectral method: w_j = sqrt(2) (z_j1/l1,
// z_j2/l2) has the normal law whose characteristic function is the
// covariance, phi_j = 2 pi u_j), kappa = 0.1 + exp(beta).  Each term is a
// plane wave, so along a column of centroids it is c_k = cos(theta_0 + k a)
// with a = w_j2 h: one thread walks a strip of GF_RY rows of one column with
// one sincos per term and a three-operation recurrence per row, Reinsch's
// form of the cosine recurrence (d_{k+1} = d_k + lambda c_k, c_{k+1} = c_k +
// d_{k+1}, lambda = -4 sin^2(a/2), d_1 = -2 sin(a/2) sin(theta_0 + a/2)),
// which stays accurate as a -> 0 where the three-term form
// c_{k+1} = 2 cos(a) c_k - c_{k-1} loses digits.  The angle is first reduced
// to [-pi/2, pi/2]: with a = a' + pi (mod 2 pi), c_k = (-1)^k cos(theta_0 +
// k a'), so such terms run the same recurrence on a' and add the odd rows
// with a minus sign.  beta stays within 2.5e-14 of the direct cosines at 256
// terms and 64-row strips.  A workgroup covers 64 columns x 4 strips of one
// sample; the sample's terms are staged in LDS.
//
// Local KL (host): the patch covariance exp(-dx^2/l1^2 - dy^2/l2^2) on the
// m x m centroids is the Kronecker product of two m x m matrices, so its
// eigenpairs are the products of the one-dimensional ones (cyclic Jacobi);
// the K largest products give mu_k and the modes v_k = vy (x) vx.
//
// kl_project_kernel: one wavefront per (sample, element), four per workgroup:
// xi_k = v_k . beta / sqrt(mu_k), lanes over the values of the element or of
// its oversampled patch (side m + 2o, Sec. 2.2, the domain on which Sec. 5.3
// takes the local KL), the
// partial sums combined by a butterfly of lane shuffles (a fixed order);
// pairs with |xi_k| > box for some k are flagged and counted.
// kl_blocks_kernel: kappa of the first K' terms on every pair's block,
// 0.1 + exp(sum_k sqrt(mu_k) xi_k v_k), one thread per element.
#include <cmath>
#include <vector>

#include "common.h"

namespace stomsfem {

constexpr int GF_TX = 64;     // columns per workgroup, one per lane
constexpr int GF_SY = 4;      // strips per workgroup, one per wavefront
constexpr int GF_RY = 64;     // rows per strip
constexpr int GF_JMAX = 1024;  // spectral terms per sample
constexpr int KL_KMAX = 16;    // local KL terms

__global__ __launch_bounds__(256) void gauss_field_kernel(int64_t nsamples, int nfine, int J,
                                                          const double* __restrict__ z,
                                                          const double* __restrict__ u, double l1, double l2,
                                                          double* __restrict__ beta, double* __restrict__ kappa,
                                                          int tiles_x, int tiles_y) {
  __shared__ double2 ws[GF_JMAX];   // (w1, w2)
  __shared__ double2 hs[GF_JMAX];   // (sin a'/2, cos a'/2), a' = w2 h reduced to [-pi/2, pi/2]
  __shared__ double2 ps[GF_JMAX];   // (phi, sign of the odd rows)
  const int64_t tiles = (int64_t)tiles_x * tiles_y;
  const int64_t nblk = nsamples * tiles;
  const double h = 1.0 / nfine, amp = sqrt(2.0 / J);
  const int lane = threadIdx.x & 63, strip = threadIdx.x >> 6;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int64_t s = b / tiles;
    const int tt = (int)(b - s * tiles);
    const int tx = tt % tiles_x, ty = tt / tiles_x;
    __syncthreads();  // the previous tile's readers are done
    for (int j = threadIdx.x; j < J; j += 256) {
      const double w1 = sqrt(2.0) * z[(s * J + j) * 2] / l1;
      const double w2 = sqrt(2.0) * z[(s * J + j) * 2 + 1] / l2;
      const double al = remainder(w2 * h, 2.0 * M_PI);  // [-pi, pi]
      const bool alt = fabs(al) > 0.5 * M_PI;
      const double alp = alt ? al - copysign(M_PI, al) : al;
      double snh, csh;
      sincos(0.5 * alp, &snh, &csh);
      ws[j] = make_double2(w1, w2);
      hs[j] = make_double2(snh, csh);
      ps[j] = make_double2(2.0 * M_PI * u[s * J + j], alt ? -1.0 : 1.0);
    }
    __syncthreads();
    const int ix = tx * GF_TX + lane, iy0 = (ty * GF_SY + strip) * GF_RY;
    const double x = (ix + 0.5) * h, y0 = (iy0 + 0.5) * h;
    double acc[GF_RY];
#pragma unroll
    for (int k = 0; k < GF_RY; ++k) acc[k] = 0.0;
    for (int j = 0; j < J; ++j) {
      const double2 w = ws[j], hh = hs[j], pp = ps[j];
      double c, sn;
      sincos(w.x * x + w.y * y0 + pp.x, &sn, &c);
      acc[0] += c;
      const double lam = -4.0 * hh.x * hh.x;
      double d = -2.0 * hh.x * (sn * hh.y + c * hh.x);
#pragma unroll
      for (int k = 1; k < GF_RY; ++k) {
        c += d;
        acc[k] = (k & 1) ? __builtin_fma(pp.y, c, acc[k]) : acc[k] + c;
        d = __builtin_fma(lam, c, d);
      }
    }
    if (ix < nfine) {
#pragma unroll
      for (int k = 0; k < GF_RY; ++k) {
        const int iy = iy0 + k;
        if (iy < nfine) {
          const double bv = amp * acc[k];
          const int64_t o = (s * nfine + iy) * (int64_t)nfine + ix;
          if (beta) beta[o] = bv;
          kappa[o] = 0.1 + exp(bv);
        }
      }
    }
  }
}

hipError_t launch_gauss_field(int64_t nsamples, int nfine, int J, const double* z, const double* u, double l1,
                              double l2, double* beta, double* kappa, hipStream_t st) {
  if (J < 1 || J > GF_JMAX) return hipErrorInvalidValue;
  const int tiles_x = (nfine + GF_TX - 1) / GF_TX, tiles_y = (nfine + GF_SY * GF_RY - 1) / (GF_SY * GF_RY);
  int64_t blocks = nsamples * (int64_t)tiles_x * tiles_y;
  if (blocks == 0) return hipSuccess;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  hipLaunchKernelGGL(gauss_field_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nsamples, nfine, J, z, u, l1, l2,
                     beta, kappa, tiles_x, tiles_y);
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

constexpr int KL_WPB = 4;  // pairs (wavefronts) per workgroup

// First fine cell (one axis) of the patch of coarse element k: the element
// widened by o cells on each side (Sec. 2.2), moved inside [0, nf) where it
// would stick out, so every patch has side m + 2o.
__device__ __forceinline__ int kl_patch_origin(int k, int m, int o, int nf) {
  const int x0 = k * m - o, hi = nf - (m + 2 * o);
  return x0 > hi ? hi : (x0 < 0 ? 0 : x0);
}

// KT: compile-time bound on K (the loops over the terms are unrolled to it)
template <int KT>
__global__ __launch_bounds__(64 * KL_WPB) void kl_project_kernel(int64_t npairs, int nc, int m, int o, int K,
                                                                 const double* __restrict__ beta,
                                                                 const double* __restrict__ mu,
                                                                 const double* __restrict__ modes, double box,
                                                                 double* __restrict__ xi,
                                                                 int32_t* __restrict__ outside,
                                                                 unsigned long long* count) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * KL_WPB + (threadIdx.x >> 6);
  if (p >= npairs) return;  // whole wavefronts only; the kernel has no barrier
  // 32-bit index arithmetic (the launch bounds npairs below 2^32)
  const uint32_t M = (uint32_t)nc * (uint32_t)nc, pu = (uint32_t)p;
  const int64_t s = pu / M;
  const int K0 = (int)(pu - (uint32_t)s * M), kx = K0 % nc, ky = K0 / nc;
  const int P = m + 2 * o;  // patch side (the element itself when o = 0)
  const int64_t nf = (int64_t)nc * m, mm = (int64_t)P * P;
  const double* B = beta + s * nf * nf + (int64_t)kl_patch_origin(ky, m, o, (int)nf) * nf +
                    kl_patch_origin(kx, m, o, (int)nf);
  double acc[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) acc[k] = 0.0;
  // lanes as rpi rows of cw columns of the patch (one division per lane)
  const int cw = P < 64 ? P : 64, rpi = 64 / cw;
  const int c0 = lane % cw, r0 = lane / cw;
  if (r0 < rpi) {
    // four rows per step so that a wavefront has four loads in flight
    constexpr int U = 4;
    for (int rb = r0; rb < P; rb += U * rpi) {
      double bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = rb + u * rpi;
        bv[u] = (r < P && c0 < P) ? B[(int64_t)r * nf + c0] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = rb + u * rpi;
        if (r < P) {
#pragma unroll
          for (int k = 0; k < KT; ++k)
            if (k < K) acc[k] += bv[u] * modes[k * mm + r * P + c0];
        }
      }
      // columns beyond the first 64 (elements wider than a wavefront)
      for (int c = c0 + cw; c < P; c += cw)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int r = rb + u * rpi;
          if (r < P) {
            const double b = B[(int64_t)r * nf + c];
#pragma unroll
            for (int k = 0; k < KT; ++k)
              if (k < K) acc[k] += b * modes[k * mm + r * P + c];
          }
        }
    }
  }
  // butterfly over the 64 lanes (a fixed order; every lane ends with the
  // sums), then lane k scales term k: one divide per wavefront
  double tk = 0.0;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    if (k < K) {
      double t = acc[k];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
      tk = lane == k ? t : tk;
    }
  }
  bool mine_out = false;
  if (lane < K) {
    const double x = tk / sqrt(mu[lane]);
    xi[p * K + lane] = x;
    mine_out = !(fabs(x) <= box);
  }
  const bool out = __any(mine_out);
  if (lane == 0) {
    if (outside) outside[p] = out ? 1 : 0;
    if (out && count) atomicAdd(count, 1ull);
  }
}

// Patches of side <= 16 (U = 4) or <= 32 (U = 16): every row of a lane's
// column in one step of U rows;
// persistent wavefronts that keep their lane's mode values in registers and
// take pairs p = w, w + (number of wavefronts), ...  The same products and
// sums in the same order as kl_project_kernel.
template <int KT, int U>
__global__ __launch_bounds__(64 * KL_WPB) void kl_project_small_kernel(int64_t npairs, int nc, int m, int o, int K,
                                                                       const double* __restrict__ beta,
                                                                       const double* __restrict__ mu,
                                                                       const double* __restrict__ modes, double box,
                                                                       double* __restrict__ xi,
                                                                       int32_t* __restrict__ outside,
                                                                       unsigned long long* count) {
  const int lane = threadIdx.x & 63;
  const int P = m + 2 * o;
  const int64_t nf = (int64_t)nc * m, mm = (int64_t)P * P;
  const int rpi = 64 / P, c0 = lane % P, r0 = lane / P;
  bool rok[U];
  int64_t roff[U];
  double mv[U][KT];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = r0 + u * rpi;
    rok[u] = r0 < rpi && r < P;
    roff[u] = rok[u] ? (int64_t)r * nf + c0 : 0;
#pragma unroll
    for (int k = 0; k < KT; ++k) mv[u][k] = (rok[u] && k < K) ? modes[k * mm + r * P + c0] : 0.0;
  }
  const double sq = lane < K ? sqrt(mu[lane]) : 1.0;
  const uint32_t M = (uint32_t)nc * (uint32_t)nc;
  const int64_t nw = (int64_t)gridDim.x * KL_WPB;
  for (int64_t p = (int64_t)blockIdx.x * KL_WPB + (threadIdx.x >> 6); p < npairs; p += nw) {
    const uint32_t pu = (uint32_t)p;
    const int64_t s = pu / M;
    const int K0 = (int)(pu - (uint32_t)s * M), kx = K0 % nc, ky = K0 / nc;
    const double* B = beta + s * nf * nf + (int64_t)kl_patch_origin(ky, m, o, (int)nf) * nf +
                      kl_patch_origin(kx, m, o, (int)nf);
    double bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) bv[u] = rok[u] ? B[roff[u]] : 0.0;
    double acc[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) acc[k] = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (rok[u]) {
#pragma unroll
        for (int k = 0; k < KT; ++k)
          if (k < K) acc[k] += bv[u] * mv[u][k];
      }
    double tk = 0.0;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < K) {
        double t = acc[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
        tk = lane == k ? t : tk;
      }
    }
    bool mine_out = false;
    if (lane < K) {
      const double x = tk / sq;
      xi[p * K + lane] = x;
      mine_out = !(fabs(x) <= box);
    }
    const bool out = __any(mine_out);
    if (lane == 0) {
      if (outside) outside[p] = out ? 1 : 0;
      if (out && count) atomicAdd(count, 1ull);
    }
  }
}

hipError_t launch_kl_project(int64_t npairs, int nc, int m, int o, int K, const double* beta, const double* mu,
                             const double* modes, double box, double* xi, int32_t* outside,
                             unsigned long long* count, hipStream_t st) {
  if (npairs == 0) return hipSuccess;
  if (K < 1 || K > KL_KMAX || o < 0 || m + 2 * o > nc * m) return hipErrorInvalidValue;
  if (npairs > 0xffffffffLL) return hipErrorInvalidValue;
  const int64_t nb = (npairs + KL_WPB - 1) / KL_WPB;
  const unsigned nbp = (unsigned)(nb < 2048 ? nb : 2048);  // persistent: about eight wavefronts per CU
  if (K <= 4 && m + 2 * o <= 16) {
    hipLaunchKernelGGL((kl_project_small_kernel<4, 4>), dim3(nbp), dim3(64 * KL_WPB), 0, st, npairs, nc, m, o, K,
                       beta, mu, modes, box, xi, outside, count);
  } else if (K <= 4 && m + 2 * o <= 32) {
    hipLaunchKernelGGL((kl_project_small_kernel<4, 16>), dim3(nbp), dim3(64 * KL_WPB), 0, st, npairs, nc, m, o, K,
                       beta, mu, modes, box, xi, outside, count);
  } else if (K <= 4)
    hipLaunchKernelGGL(kl_project_kernel<4>, dim3((unsigned)nb), dim3(64 * KL_WPB), 0, st, npairs, nc, m, o, K, beta,
                       mu, modes, box, xi, outside, count);
  else
    hipLaunchKernelGGL(kl_project_kernel<KL_KMAX>, dim3((unsigned)nb), dim3(64 * KL_WPB), 0, st, npairs, nc, m, o, K,
                       beta, mu, modes, box, xi, outside, count);
  return hipGetLastError();
}

// ---- oversampled patches in 3 x 3-element meshes ----
// The oversampled Petrov-Galerkin stiffness of an element depends only on
// the coefficient of its patch (side P = m + 2o) and on where the element
// sits in it: at offset 0, o or 2o along each axis (class 0, 1, 2; the patch
// is moved inside the domain at the edge; 1 <= o <= m).  A 3 x 3-element
// mesh has one element of every class, so a patch placed there at that
// element's patch origin (the rest of the mesh 1, never read by the cell
// problems) gives the element's stiffness through the ordinary oversampling
// kernels.  embed_patch_kernel: item i of fields [count][3m][3m] takes
// blocks[i] ([P][P]) at class (cx, cy).
__global__ __launch_bounds__(256) void embed_patch_kernel(int64_t count, int m, int o, int cx, int cy,
                                                          const double* __restrict__ blocks,
                                                          double* __restrict__ fields) {
  const int P = m + 2 * o, n3 = 3 * m;
  const int64_t per = (int64_t)n3 * n3;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= count * per) return;
  const int64_t i = t / per;
  const int e = (int)(t - i * per), y = e / n3, x = e - (e / n3) * n3;
  const int x0 = kl_patch_origin(cx, m, o, n3), y0 = kl_patch_origin(cy, m, o, n3);
  const bool in = x >= x0 && x < x0 + P && y >= y0 && y < y0 + P;
  fields[t] = in ? blocks[i * (int64_t)P * P + (int64_t)(y - y0) * P + (x - x0)] : 1.0;
}

// The class element's 16 entries of each 3 x 3 mesh (S9 [count][9][16],
// st9 [count][9]) into dst [count][16] and its status into dst_status [count].
__global__ __launch_bounds__(256) void pick_class_kernel(int64_t count, int cx, int cy, const double* __restrict__ S9,
                                                         const int32_t* __restrict__ st9, double* __restrict__ dst,
                                                         int32_t* __restrict__ dst_status) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const int e = cy * 3 + cx;
#pragma unroll
  for (int q = 0; q < 16; ++q) dst[i * 16 + q] = S9[(i * 9 + e) * 16 + q];
  dst_status[i] = st9[i * 9 + e];
}

hipError_t launch_embed_patch(int64_t count, int m, int o, int cx, int cy, const double* blocks, double* fields,
                              hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (o < 1 || o > m || cx < 0 || cx > 2 || cy < 0 || cy > 2) return hipErrorInvalidValue;
  const int64_t n = count * 9 * (int64_t)m * m;
  const int64_t nb = (n + 255) / 256;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(embed_patch_kernel, dim3((unsigned)nb), dim3(256), 0, st, count, m, o, cx, cy, blocks, fields);
  return hipGetLastError();
}

hipError_t launch_pick_class(int64_t count, int cx, int cy, const double* S9, const int32_t* st9, double* dst,
                             int32_t* dst_status, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (cx < 0 || cx > 2 || cy < 0 || cy > 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pick_class_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, cx, cy, S9,
                     st9, dst, dst_status);
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
