/*
 * CPU FP64 oracle for the stochastic multiscale FEM (Hou, Li & Zhang,
 * "Exploring the locally low dimensional structure in solving random
 * elliptic PDEs").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links, includes or calls anything here, and nothing here is shared with it.
 *
 * Everything is double precision, plain loops, no blocking or fusion:
 *   - Q1 element stiffness from its definition (2x2 Gauss quadrature of the
 *     bilinear shape-function gradients, exact for these polynomials);
 *   - the cell problems of the MsFEM basis (Sec. 2.2, eq. MsFEB): all L = 4
 *     Dirichlet problems are solved (no partition-of-unity shortcut) with a
 *     textbook banded Cholesky (Cholesky-Crout, left looking);
 *   - the upscaled stiffness by the element-sum form of eq. stiffness_local;
 *   - oversampling (remark in Sec. 2.2): cell problems on an enlarged patch,
 *     the basis re-normalised to nodal values on K, and the Petrov-Galerkin
 *     stiffness of eq. stiffness_local_petrov with bilinear test functions;
 *     its non-symmetric coarse system by banded LU with partial pivoting;
 *   - coarse assembly and solve of S U = b (eq. upscaleSUF), Petrov-Galerkin
 *     load (eq. stiffness_local_petrov) for f = 1;
 *   - the Monte Carlo mean and variance of the coarse solution (Sec. 4.1.1);
 *   - a global fine-grid Q1 FEM (brute force, for small meshes only);
 *   - the coefficient generator of the synthetic workloads.
 *
 * Conventions.  Coefficient arrays are piecewise constant per fine element,
 * sampled at the element centroid, row-major a[iy][ix] (iy = y index).  A
 * coarse element K = (kx, ky) has index ky*ncx + kx.  Its local nodes are
 * numbered counter-clockwise from the lower-left corner: 0=(x0,y0),
 * 1=(x1,y0), 2=(x1,y1), 3=(x0,y1).  The 10 unique entries of the symmetric
 * 4x4 upscaled stiffness are packed as 00,01,02,03,11,12,13,22,23,33.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENOTSPD -4

/* ------------------------------------------------------------------------ */
/* Q1 element stiffness for a unit coefficient on a square element.          */
/* ------------------------------------------------------------------------ */

/* Bilinear shape functions on the reference square [0,1]^2, CCW numbering. */
static void q1_grad(double x, double y, double gx[4], double gy[4]) {
  gx[0] = -(1.0 - y); gy[0] = -(1.0 - x);
  gx[1] = (1.0 - y);  gy[1] = -x;
  gx[2] = y;          gy[2] = x;
  gx[3] = -y;         gy[3] = (1.0 - x);
}

/* K_ref[a][b] = int_{[0,1]^2} grad N_a . grad N_b.  In 2-D this does not
 * depend on the element size.  2x2 Gauss-Legendre is exact (degree 2). */
void orc_q1_kref(double K[16]) {
  const double g = 0.5 / sqrt(3.0);
  const double pts[2] = {0.5 - g, 0.5 + g};
  memset(K, 0, 16 * sizeof(double));
  for (int qi = 0; qi < 2; ++qi)
    for (int qj = 0; qj < 2; ++qj) {
      double gx[4], gy[4];
      q1_grad(pts[qi], pts[qj], gx, gy);
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) K[4 * a + b] += 0.25 * (gx[a] * gx[b] + gy[a] * gy[b]);
    }
}

static double KREF[16];
static int kref_ready = 0;
static void ensure_kref(void) {
  if (!kref_ready) {
    orc_q1_kref(KREF);
    kref_ready = 1;
  }
}

/* ------------------------------------------------------------------------ */
/* Banded Cholesky (lower band storage B[i*(bw+1)+d] = A(i, i-d)).           */
/* ------------------------------------------------------------------------ */

#define BAND(B, bw, i, j) (B)[(size_t)(i) * ((bw) + 1) + ((i) - (j))]

/* In place: on return the band holds L with A = L L^T.  Returns 0 or the
 * negative (1-based) index of the first non-positive pivot. */
int orc_band_chol(int n, int bw, double* B) {
  for (int j = 0; j < n; ++j) {
    double s = BAND(B, bw, j, j);
    int k0 = j - bw > 0 ? j - bw : 0;
    for (int k = k0; k < j; ++k) s -= BAND(B, bw, j, k) * BAND(B, bw, j, k);
    if (!(s > 0.0)) return -(j + 1);
    double ljj = sqrt(s);
    BAND(B, bw, j, j) = ljj;
    int i1 = j + bw < n - 1 ? j + bw : n - 1;
    for (int i = j + 1; i <= i1; ++i) {
      double t = BAND(B, bw, i, j);
      int kk0 = i - bw > 0 ? i - bw : 0;
      for (int k = kk0; k < j; ++k) t -= BAND(B, bw, i, k) * BAND(B, bw, j, k);
      BAND(B, bw, i, j) = t / ljj;
    }
  }
  return 0;
}

/* Solve L L^T x = b in place for nrhs right-hand sides stored x[r*n + i]. */
void orc_band_solve(int n, int bw, const double* L, int nrhs, double* x) {
  for (int r = 0; r < nrhs; ++r) {
    double* v = x + (size_t)r * n;
    for (int i = 0; i < n; ++i) {
      double t = v[i];
      int k0 = i - bw > 0 ? i - bw : 0;
      for (int k = k0; k < i; ++k) t -= BAND(L, bw, i, k) * v[k];
      v[i] = t / BAND(L, bw, i, i);
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = v[i];
      int k1 = i + bw < n - 1 ? i + bw : n - 1;
      for (int k = i + 1; k <= k1; ++k) t -= BAND(L, bw, k, i) * v[k];
      v[i] = t / BAND(L, bw, i, i);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Cell problems (eq. MsFEB) on one coarse element with m x m fine cells.     */
/* ------------------------------------------------------------------------ */

enum { ORC_BC_LINEAR = 0, ORC_BC_OSC = 1 };

/* Boundary data g^l at every node of the (m+1)^2 local grid (interior nodes
 * are left at 0).  Linear BC: the bilinear nodal function p^l.  Oscillatory
 * BC: on each edge the 1-D discrete harmonic profile of the edge-adjacent
 * fine elements, running from 1 at corner l to 0 at the other end (a reading
 * of the option named in Sec. 5.3; with a constant coefficient it reduces to
 * the linear data). */
static void cell_boundary_data(int m, const double* a, ptrdiff_t lda, int bc, double* g /*[4][(m+1)^2]*/) {
  const int nn = m + 1;
  memset(g, 0, sizeof(double) * 4 * (size_t)nn * nn);
  if (bc == ORC_BC_LINEAR) {
    for (int py = 0; py <= m; ++py)
      for (int px = 0; px <= m; ++px) {
        if (px != 0 && px != m && py != 0 && py != m) continue;
        double x = (double)px / m, y = (double)py / m;
        int id = py * nn + px;
        g[0 * nn * nn + id] = (1.0 - x) * (1.0 - y);
        g[1 * nn * nn + id] = x * (1.0 - y);
        g[2 * nn * nn + id] = x * y;
        g[3 * nn * nn + id] = (1.0 - x) * y;
      }
    return;
  }
  /* oscillatory: resistances along each edge */
  double* u = (double*)malloc(sizeof(double) * (m + 1));
  double* k = (double*)malloc(sizeof(double) * m);
  /* edge 0: bottom, from corner 0 (px=0) to corner 1 (px=m); element row 0 */
  /* edge 1: right,  from corner 1 (py=0) to corner 2 (py=m); element col m-1 */
  /* edge 2: top,    from corner 3 (px=0) to corner 2 (px=m); element row m-1 */
  /* edge 3: left,   from corner 0 (py=0) to corner 3 (py=m); element col 0 */
  for (int e = 0; e < 4; ++e) {
    for (int s = 0; s < m; ++s) {
      if (e == 0) k[s] = a[0 * lda + s];
      if (e == 1) k[s] = a[(ptrdiff_t)s * lda + (m - 1)];
      if (e == 2) k[s] = a[(ptrdiff_t)(m - 1) * lda + s];
      if (e == 3) k[s] = a[(ptrdiff_t)s * lda + 0];
    }
    double tot = 0.0;
    for (int s = 0; s < m; ++s) tot += 1.0 / k[s];
    /* u(t) = sum_{s >= t} (1/k_s) / sum_s (1/k_s): 1 at t = 0, 0 at t = m */
    for (int t = 0; t <= m; ++t) {
      double r = 0.0;
      for (int s = t; s < m; ++s) r += 1.0 / k[s];
      u[t] = r / tot;
    }
    for (int t = 0; t <= m; ++t) {
      int id;
      int lo, hi; /* corner at t = 0 gets u, corner at t = m gets 1 - u */
      if (e == 0) { id = 0 * nn + t; lo = 0; hi = 1; }
      else if (e == 1) { id = t * nn + m; lo = 1; hi = 2; }
      else if (e == 2) { id = m * nn + t; lo = 3; hi = 2; }
      else { id = t * nn + 0; lo = 0; hi = 3; }
      g[lo * nn * nn + id] = u[t];
      g[hi * nn * nn + id] = 1.0 - u[t];
    }
  }
  free(u);
  free(k);
}

/* Solve the four cell problems.  phi[l][(m+1)^2] receives the full nodal
 * field (boundary data included).  Returns 0, ORC_ENOTSPD or ORC_ENOMEM. */
int orc_cell_phi(int m, const double* a, ptrdiff_t lda, int bc, double* phi) {
  ensure_kref();
  if (m < 1) return ORC_EINVAL;
  const int nn = m + 1, ni = m - 1, nI = ni * ni, bw = m;
  double* g = phi; /* boundary data written straight into the output */
  cell_boundary_data(m, a, lda, bc, g);
  if (nI == 0) return ORC_OK;
  double* B = (double*)calloc((size_t)nI * (bw + 1), sizeof(double));
  double* rhs = (double*)calloc((size_t)4 * nI, sizeof(double));
  if (!B || !rhs) {
    free(B);
    free(rhs);
    return ORC_ENOMEM;
  }
  /* assemble K_II (lower band) and rhs^l = -K_IB g^l element by element */
  for (int ey = 0; ey < m; ++ey)
    for (int ex = 0; ex < m; ++ex) {
      double ae = a[(ptrdiff_t)ey * lda + ex];
      int px[4] = {ex, ex + 1, ex + 1, ex};
      int py[4] = {ey, ey, ey + 1, ey + 1};
      for (int al = 0; al < 4; ++al) {
        int ia = (px[al] > 0 && px[al] < m && py[al] > 0 && py[al] < m) ? (py[al] - 1) * ni + (px[al] - 1) : -1;
        if (ia < 0) continue;
        for (int be = 0; be < 4; ++be) {
          double kab = ae * KREF[4 * al + be];
          int ib = (px[be] > 0 && px[be] < m && py[be] > 0 && py[be] < m) ? (py[be] - 1) * ni + (px[be] - 1) : -1;
          if (ib >= 0) {
            if (ib <= ia) BAND(B, bw, ia, ib) += kab;
          } else {
            int nid = py[be] * nn + px[be];
            for (int l = 0; l < 4; ++l) rhs[(size_t)l * nI + ia] -= kab * g[(size_t)l * nn * nn + nid];
          }
        }
      }
    }
  int st = orc_band_chol(nI, bw, B);
  if (st != 0) {
    free(B);
    free(rhs);
    return ORC_ENOTSPD;
  }
  orc_band_solve(nI, bw, B, 4, rhs);
  for (int l = 0; l < 4; ++l)
    for (int iy = 0; iy < ni; ++iy)
      for (int ix = 0; ix < ni; ++ix)
        phi[(size_t)l * nn * nn + (iy + 1) * nn + (ix + 1)] = rhs[(size_t)l * nI + iy * ni + ix];
  free(B);
  free(rhs);
  return ORC_OK;
}

/* S_ll' = sum_e a_e phi^l_e^T K_ref phi^l'_e  (element sum of eq. stiffness_local).
 * If test != NULL the second factor is replaced by test[l'] (Petrov-Galerkin
 * form of eq. stiffness_local_petrov). */
void orc_energy_S(int m, const double* a, ptrdiff_t lda, const double* phi, const double* test, double S[16]) {
  ensure_kref();
  const int nn = m + 1;
  const double* psi = test ? test : phi;
  memset(S, 0, 16 * sizeof(double));
  for (int ey = 0; ey < m; ++ey)
    for (int ex = 0; ex < m; ++ex) {
      double ae = a[(ptrdiff_t)ey * lda + ex];
      int nid[4] = {ey * nn + ex, ey * nn + ex + 1, (ey + 1) * nn + ex + 1, (ey + 1) * nn + ex};
      for (int l = 0; l < 4; ++l)
        for (int lp = 0; lp < 4; ++lp) {
          double s = 0.0;
          for (int al = 0; al < 4; ++al)
            for (int be = 0; be < 4; ++be)
              s += phi[(size_t)l * nn * nn + nid[al]] * KREF[4 * al + be] * psi[(size_t)lp * nn * nn + nid[be]];
          S[4 * l + lp] += ae * s;
        }
    }
}

/* Galerkin load b_l = int_K f phi^l for a constant f: the Q1 interpolant of
 * phi^l is integrated exactly, i.e. (h^2/4) * sum over element corners. */
void orc_galerkin_load(int m, double H, double f, const double* phi, double b[4]) {
  const int nn = m + 1;
  const double h = H / m;
  for (int l = 0; l < 4; ++l) {
    double s = 0.0;
    for (int ey = 0; ey < m; ++ey)
      for (int ex = 0; ex < m; ++ex) {
        int nid[4] = {ey * nn + ex, ey * nn + ex + 1, (ey + 1) * nn + ex + 1, (ey + 1) * nn + ex};
        for (int c = 0; c < 4; ++c) s += phi[(size_t)l * nn * nn + nid[c]];
      }
    b[l] = f * h * h * 0.25 * s;
  }
}

static const int PACK_I[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
static const int PACK_J[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

/* Upscaled stiffness of one coarse element: packed[10].  pu_err (optional)
 * receives max |sum_l phi^l - 1| over the nodes. */
int orc_cell_S(int m, const double* a, ptrdiff_t lda, int bc, double* packed, double* pu_err) {
  const int nn = m + 1;
  double* phi = (double*)malloc(sizeof(double) * 4 * (size_t)nn * nn);
  if (!phi) return ORC_ENOMEM;
  int st = orc_cell_phi(m, a, lda, bc, phi);
  if (st == ORC_OK) {
    double S[16];
    orc_energy_S(m, a, lda, phi, NULL, S);
    for (int q = 0; q < 10; ++q) packed[q] = S[4 * PACK_I[q] + PACK_J[q]];
    if (pu_err) {
      double e = 0.0;
      for (int i = 0; i < nn * nn; ++i) {
        double s = phi[i] + phi[nn * nn + i] + phi[2 * nn * nn + i] + phi[3 * nn * nn + i] - 1.0;
        if (fabs(s) > e) e = fabs(s);
      }
      *pu_err = e;
    }
  }
  free(phi);
  return st;
}

/* All (coarse element, sample) pairs.  a: [N][ncy*m][ncx*m]; S: [N][ncy*ncx][10];
 * status (optional): [N][ncy*ncx].  Returns the first non-OK status seen. */
int orc_upscale(int64_t N, int ncx, int ncy, int m, const double* a, int bc, double* S, int32_t* status,
                double* pu_err_max, int nthreads) {
  if (N < 0 || ncx < 1 || ncy < 1 || m < 1 || !a || !S) return ORC_EINVAL;
  const int64_t M = (int64_t)ncx * ncy;
  const ptrdiff_t lda = (ptrdiff_t)ncx * m;
  const int64_t per_sample = (int64_t)ncy * m * lda;
  int worst = ORC_OK;
  double pu = 0.0;
  ensure_kref();
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads) reduction(max : pu) reduction(min : worst)
#endif
  for (int64_t t = 0; t < N * M; ++t) {
    int64_t s = t / M;
    int K = (int)(t % M);
    int kx = K % ncx, ky = K / ncx;
    const double* blk = a + s * per_sample + (ptrdiff_t)ky * m * lda + (ptrdiff_t)kx * m;
    double e = 0.0;
    int st = orc_cell_S(m, blk, lda, bc, S + t * 10, &e);
    if (status) status[t] = st;
    if (st < worst) worst = st;
    if (e > pu) pu = e;
  }
  if (pu_err_max) *pu_err_max = pu;
  return worst;
}

/* ------------------------------------------------------------------------ */
/* Coarse system S U = b (eq. upscaleSUF), zero Dirichlet data.              */
/* ------------------------------------------------------------------------ */

/* One sample.  Sk: [M][10]; load: [M][4] element loads, or NULL for f = 1
 * with the Petrov-Galerkin load int_K f p^l = H^2/4 (H = 1/ncx). */
int orc_coarse_one(int ncx, int ncy, const double* Sk, const double* load, double* U) {
  const int nix = ncx - 1, niy = ncy - 1, nU = nix * niy, bw = ncx;
  if (nU <= 0) return ORC_OK;
  double* B = (double*)calloc((size_t)nU * (bw + 1), sizeof(double));
  double* b = (double*)calloc((size_t)nU, sizeof(double));
  if (!B || !b) {
    free(B);
    free(b);
    return ORC_ENOMEM;
  }
  const double H = 1.0 / ncx;
  for (int ky = 0; ky < ncy; ++ky)
    for (int kx = 0; kx < ncx; ++kx) {
      int K = ky * ncx + kx;
      double S4[16];
      for (int q = 0; q < 10; ++q) {
        S4[4 * PACK_I[q] + PACK_J[q]] = Sk[(size_t)K * 10 + q];
        S4[4 * PACK_J[q] + PACK_I[q]] = Sk[(size_t)K * 10 + q];
      }
      int px[4] = {kx, kx + 1, kx + 1, kx};
      int py[4] = {ky, ky, ky + 1, ky + 1};
      for (int al = 0; al < 4; ++al) {
        int ia = (px[al] > 0 && px[al] < ncx && py[al] > 0 && py[al] < ncy) ? (py[al] - 1) * nix + (px[al] - 1) : -1;
        if (ia < 0) continue;
        b[ia] += load ? load[(size_t)K * 4 + al] : 0.25 * H * H;
        for (int be = 0; be < 4; ++be) {
          int ib = (px[be] > 0 && px[be] < ncx && py[be] > 0 && py[be] < ncy) ? (py[be] - 1) * nix + (px[be] - 1) : -1;
          if (ib >= 0 && ib <= ia) BAND(B, bw, ia, ib) += S4[4 * al + be];
        }
      }
    }
  int st = orc_band_chol(nU, bw, B);
  if (st == 0) {
    orc_band_solve(nU, bw, B, 1, b);
    memcpy(U, b, sizeof(double) * nU);
  }
  free(B);
  free(b);
  return st == 0 ? ORC_OK : ORC_ENOTSPD;
}

/* All samples, then the Monte Carlo estimates of Sec. 4.1.1:
 * mean = (1/N) sum U, var = (1/N) sum U^2 - mean^2 (both optional). */
int orc_coarse_solve(int ncx, int ncy, int64_t N, const double* S, const double* load, double* U,
                     double* qoi_mean, double* qoi_var, int32_t* status, int nthreads) {
  if (ncx < 1 || ncy < 1 || N < 0 || !S || !U) return ORC_EINVAL;
  const int64_t M = (int64_t)ncx * ncy;
  const int nU = (ncx - 1) * (ncy - 1);
  int worst = ORC_OK;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(min : worst)
#endif
  for (int64_t s = 0; s < N; ++s) {
    int st = orc_coarse_one(ncx, ncy, S + s * M * 10, load, U + s * nU);
    if (status) status[s] = st;
    if (st < worst) worst = st;
  }
  if (qoi_mean || qoi_var) {
    for (int i = 0; i < nU; ++i) {
      double m1 = 0.0, m2 = 0.0;
      for (int64_t s = 0; s < N; ++s) {
        double u = U[s * nU + i];
        m1 += u;
        m2 += u * u;
      }
      m1 = N > 0 ? m1 / (double)N : 0.0;
      m2 = N > 0 ? m2 / (double)N : 0.0;
      if (qoi_mean) qoi_mean[i] = m1;
      if (qoi_var) qoi_var[i] = m2 - m1 * m1;
    }
  }
  return worst;
}

/* ------------------------------------------------------------------------ */
/* Oversampling with the Petrov-Galerkin local stiffness (Sec. 2.2, remark   */
/* on oversampling, and eq. stiffness_local_petrov).                          */
/* ------------------------------------------------------------------------ */

/* Origin (fine-cell index, one axis) of the oversampled patch of coarse
 * element k: m + 2o cells centred on the element's m cells, moved inside
 * [0, nf) where it would stick out of the domain. */
int orc_os_origin(int k, int m, int o, int nf) {
  int x0 = k * m - o;
  if (x0 > nf - (m + 2 * o)) x0 = nf - (m + 2 * o);
  if (x0 < 0) x0 = 0;
  return x0;
}

/* X = A^{-1} (4x4, row-major) by Gauss-Jordan elimination with partial
 * pivoting.  Returns ORC_EINVAL if a pivot vanishes. */
static int inv4(const double A[16], double X[16]) {
  double M[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 8; ++j) M[i][j] = j < 4 ? A[4 * i + j] : (j - 4 == i ? 1.0 : 0.0);
  for (int c = 0; c < 4; ++c) {
    int p = c;
    for (int i = c + 1; i < 4; ++i)
      if (fabs(M[i][c]) > fabs(M[p][c])) p = i;
    if (!(fabs(M[p][c]) > 0.0)) return ORC_EINVAL;
    for (int j = 0; j < 8; ++j) {
      double t = M[c][j];
      M[c][j] = M[p][j];
      M[p][j] = t;
    }
    double inv = 1.0 / M[c][c];
    for (int j = 0; j < 8; ++j) M[c][j] *= inv;
    for (int i = 0; i < 4; ++i) {
      if (i == c) continue;
      double f = M[i][c];
      for (int j = 0; j < 8; ++j) M[i][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) X[4 * i + j] = M[i][4 + j];
  return ORC_OK;
}

/* Oversampled MsFEM basis of coarse element (kx, ky) (m x m fine cells,
 * oversampling by o fine cells on each side, so the patch has m + 2o cells
 * per side; the oversampling ratio is (m + 2o)/m):
 *   1. the four cell problems (eq. MsFEB) on the patch, with the bilinear
 *      nodal functions of the patch corners as boundary data: psi^j;
 *   2. Psi[k][j] = psi^j(x_k) at the corners x_k of K (CCW from lower left);
 *   3. phi^i = sum_j C[i][j] psi^j restricted to K, with C chosen so that
 *      phi^i(x_k) = delta_ik, i.e. C Psi^T = I.
 * a: the sample's whole field [nfy][lda]; phiK: [4][(m+1)^2] on K's nodes.
 * Psi (optional): [16]. */
int orc_cell_phi_os(int m, int o, int nfx, int nfy, const double* a, ptrdiff_t lda, int kx, int ky, double* phiK,
                    double* Psi_out) {
  const int mp = m + 2 * o, nnp = mp + 1, nn = m + 1;
  if (m < 1 || o < 0 || mp > nfx || mp > nfy) return ORC_EINVAL;
  const int x0 = orc_os_origin(kx, m, o, nfx), y0 = orc_os_origin(ky, m, o, nfy);
  double* psi = (double*)malloc(sizeof(double) * 4 * (size_t)nnp * nnp);
  if (!psi) return ORC_ENOMEM;
  int st = orc_cell_phi(mp, a + (ptrdiff_t)y0 * lda + x0, lda, ORC_BC_LINEAR, psi);
  if (st != ORC_OK) {
    free(psi);
    return st;
  }
  const int cx = kx * m - x0, cy = ky * m - y0; /* K's lower-left node in patch nodes */
  const int kpx[4] = {cx, cx + m, cx + m, cx}, kpy[4] = {cy, cy, cy + m, cy + m};
  double Psi[16], PsiT[16], C[16];
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) Psi[4 * k + j] = psi[(size_t)j * nnp * nnp + kpy[k] * nnp + kpx[k]];
  if (Psi_out) memcpy(Psi_out, Psi, sizeof Psi);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) PsiT[4 * i + j] = Psi[4 * j + i];
  st = inv4(PsiT, C); /* C = (Psi^T)^{-1} */
  if (st == ORC_OK)
    for (int i = 0; i < 4; ++i)
      for (int py = 0; py <= m; ++py)
        for (int px = 0; px <= m; ++px) {
          double v = 0.0;
          for (int j = 0; j < 4; ++j) v += C[4 * i + j] * psi[(size_t)j * nnp * nnp + (cy + py) * nnp + (cx + px)];
          phiK[(size_t)i * nn * nn + py * nn + px] = v;
        }
  free(psi);
  return st;
}

/* Petrov-Galerkin upscaled stiffness of coarse element (kx, ky) with
 * oversampling: S16[l][l'] = int_K a grad phi^l . grad p^l' (row-major; l the
 * oversampled multiscale trial function, p^l' the bilinear nodal test
 * function of K), by the element sum.  o = 0 gives the MsFEM stiffness of
 * eq. stiffness_local. */
int orc_cell_S_os(int m, int o, int nfx, int nfy, const double* a, ptrdiff_t lda, int kx, int ky, double S16[16]) {
  const int nn = m + 1;
  double* phiK = (double*)malloc(sizeof(double) * 8 * (size_t)nn * nn);
  if (!phiK) return ORC_ENOMEM;
  double* pt = phiK + 4 * (size_t)nn * nn;
  int st = orc_cell_phi_os(m, o, nfx, nfy, a, lda, kx, ky, phiK, NULL);
  if (st == ORC_OK) {
    for (int py = 0; py <= m; ++py)
      for (int px = 0; px <= m; ++px) {
        const double x = (double)px / m, y = (double)py / m;
        const int id = py * nn + px;
        pt[0 * nn * nn + id] = (1.0 - x) * (1.0 - y);
        pt[1 * nn * nn + id] = x * (1.0 - y);
        pt[2 * nn * nn + id] = x * y;
        pt[3 * nn * nn + id] = (1.0 - x) * y;
      }
    orc_energy_S(m, a + (ptrdiff_t)ky * m * lda + (ptrdiff_t)kx * m, lda, phiK, pt, S16);
  }
  free(phiK);
  return st;
}

/* All pairs.  a: [N][ncy*m][ncx*m]; S16: [N][ncy*ncx][16]; status optional. */
int orc_upscale_os(int64_t N, int ncx, int ncy, int m, int o, const double* a, double* S16, int32_t* status,
                   int nthreads) {
  if (N < 0 || ncx < 1 || ncy < 1 || m < 1 || o < 0 || !a || !S16) return ORC_EINVAL;
  if (m + 2 * o > ncx * m || m + 2 * o > ncy * m) return ORC_EINVAL;
  const int64_t M = (int64_t)ncx * ncy;
  const ptrdiff_t lda = (ptrdiff_t)ncx * m;
  const int64_t per_sample = (int64_t)ncy * m * lda;
  int worst = ORC_OK;
  ensure_kref();
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads) reduction(min : worst)
#endif
  for (int64_t t = 0; t < N * M; ++t) {
    int64_t s = t / M;
    int K = (int)(t % M);
    int st = orc_cell_S_os(m, o, ncx * m, ncy * m, a + s * per_sample, lda, K % ncx, K / ncx, S16 + t * 16);
    if (status) status[t] = st;
    if (st < worst) worst = st;
  }
  return worst;
}

/* Banded LU with partial pivoting (kl sub-, ku super-diagonals; row i keeps
 * columns [i - kl, i + kl + ku], the upper band widened by kl for the row
 * interchanges) and the solve of A x = b in place.  A(i, c) at
 * W[i * (2 kl + ku + 1) + c - i + kl].  Returns 0 or ORC_ENOTSPD on a zero
 * pivot. */
#define GB(W, w, kl, i, c) (W)[(size_t)(i) * (w) + ((c) - (i) + (kl))]
int orc_band_lu_solve(int n, int kl, int ku, double* W, double* b) {
  const int w = 2 * kl + ku + 1;
  for (int j = 0; j < n; ++j) {
    int i1 = j + kl < n - 1 ? j + kl : n - 1;
    int p = j;
    for (int i = j + 1; i <= i1; ++i)
      if (fabs(GB(W, w, kl, i, j)) > fabs(GB(W, w, kl, p, j))) p = i;
    if (!(fabs(GB(W, w, kl, p, j)) > 0.0)) return ORC_ENOTSPD;
    int c1 = j + kl + ku < n - 1 ? j + kl + ku : n - 1;
    if (p != j) {
      for (int c = j; c <= c1; ++c) {
        double t = GB(W, w, kl, j, c);
        GB(W, w, kl, j, c) = GB(W, w, kl, p, c);
        GB(W, w, kl, p, c) = t;
      }
      double t = b[j];
      b[j] = b[p];
      b[p] = t;
    }
    for (int i = j + 1; i <= i1; ++i) {
      double l = GB(W, w, kl, i, j) / GB(W, w, kl, j, j);
      GB(W, w, kl, i, j) = 0.0;
      for (int c = j + 1; c <= c1; ++c) GB(W, w, kl, i, c) -= l * GB(W, w, kl, j, c);
      b[i] -= l * b[j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = b[i];
    int c1 = i + kl + ku < n - 1 ? i + kl + ku : n - 1;
    for (int c = i + 1; c <= c1; ++c) t -= GB(W, w, kl, i, c) * b[c];
    b[i] = t / GB(W, w, kl, i, i);
  }
  return ORC_OK;
}

/* One sample of the Petrov-Galerkin coarse system (eq. upscaleSUF with the
 * local quantities of eq. stiffness_local_petrov): the equation of interior
 * node a (test function a) is sum_b G[a][b] U_b = b_a with
 * G[a][b] = sum_K S16^K[l(b)][l'(a)].  S16: [M][16]; load as in
 * orc_coarse_one. */
int orc_coarse_pg_one(int ncx, int ncy, const double* S16, const double* load, double* U) {
  const int nix = ncx - 1, niy = ncy - 1, nU = nix * niy, kl = ncx, ku = ncx;
  if (nU <= 0) return ORC_OK;
  const int w = 2 * kl + ku + 1;
  double* W = (double*)calloc((size_t)nU * w, sizeof(double));
  if (!W) return ORC_ENOMEM;
  const double H = 1.0 / ncx;
  for (int i = 0; i < nU; ++i) U[i] = 0.0;
  for (int ky = 0; ky < ncy; ++ky)
    for (int kx = 0; kx < ncx; ++kx) {
      int K = ky * ncx + kx;
      int px[4] = {kx, kx + 1, kx + 1, kx};
      int py[4] = {ky, ky, ky + 1, ky + 1};
      for (int te = 0; te < 4; ++te) { /* test (row) */
        int ia = (px[te] > 0 && px[te] < ncx && py[te] > 0 && py[te] < ncy) ? (py[te] - 1) * nix + (px[te] - 1) : -1;
        if (ia < 0) continue;
        U[ia] += load ? load[(size_t)K * 4 + te] : 0.25 * H * H;
        for (int tr = 0; tr < 4; ++tr) { /* trial (column) */
          int ib = (px[tr] > 0 && px[tr] < ncx && py[tr] > 0 && py[tr] < ncy) ? (py[tr] - 1) * nix + (px[tr] - 1) : -1;
          if (ib >= 0) GB(W, w, kl, ia, ib) += S16[(size_t)K * 16 + 4 * tr + te];
        }
      }
    }
  int st = orc_band_lu_solve(nU, kl, ku, W, U);
  free(W);
  return st;
}

int orc_coarse_pg_solve(int ncx, int ncy, int64_t N, const double* S16, const double* load, double* U,
                        double* qoi_mean, double* qoi_var, int32_t* status, int nthreads) {
  if (ncx < 1 || ncy < 1 || N < 0 || !S16 || !U) return ORC_EINVAL;
  const int64_t M = (int64_t)ncx * ncy;
  const int nU = (ncx - 1) * (ncy - 1);
  int worst = ORC_OK;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(min : worst)
#endif
  for (int64_t s = 0; s < N; ++s) {
    int st = orc_coarse_pg_one(ncx, ncy, S16 + s * M * 16, load, U + s * nU);
    if (status) status[s] = st;
    if (st < worst) worst = st;
  }
  if (qoi_mean || qoi_var) {
    for (int i = 0; i < nU; ++i) {
      double m1 = 0.0, m2 = 0.0;
      for (int64_t s = 0; s < N; ++s) {
        double u = U[s * nU + i];
        m1 += u;
        m2 += u * u;
      }
      m1 = N > 0 ? m1 / (double)N : 0.0;
      m2 = N > 0 ? m2 / (double)N : 0.0;
      if (qoi_mean) qoi_mean[i] = m1;
      if (qoi_var) qoi_var[i] = m2 - m1 * m1;
    }
  }
  return worst;
}

/* ------------------------------------------------------------------------ */
/* Global fine-grid Q1 FEM on [0,1]^2 (brute force, small meshes only).       */
/* ------------------------------------------------------------------------ */

/* a: [nf][nf] per fine element; zero Dirichlet; constant source f; the load
 * int f N_i is exact for constant f: f h^2 per interior node.  u: [(nf-1)^2]. */
int orc_fine_fem(int nf, const double* a, double f, double* u) {
  ensure_kref();
  const int ni = nf - 1, nU = ni * ni, bw = nf;
  if (nU <= 0) return ORC_OK;
  double* B = (double*)calloc((size_t)nU * (bw + 1), sizeof(double));
  if (!B) return ORC_ENOMEM;
  const double h = 1.0 / nf;
  for (int i = 0; i < nU; ++i) u[i] = f * h * h;
  for (int ey = 0; ey < nf; ++ey)
    for (int ex = 0; ex < nf; ++ex) {
      double ae = a[(size_t)ey * nf + ex];
      int px[4] = {ex, ex + 1, ex + 1, ex};
      int py[4] = {ey, ey, ey + 1, ey + 1};
      for (int al = 0; al < 4; ++al) {
        int ia = (px[al] > 0 && px[al] < nf && py[al] > 0 && py[al] < nf) ? (py[al] - 1) * ni + (px[al] - 1) : -1;
        if (ia < 0) continue;
        for (int be = 0; be < 4; ++be) {
          int ib = (px[be] > 0 && px[be] < nf && py[be] > 0 && py[be] < nf) ? (py[be] - 1) * ni + (px[be] - 1) : -1;
          if (ib >= 0 && ib <= ia) BAND(B, bw, ia, ib) += ae * KREF[4 * al + be];
        }
      }
    }
  int st = orc_band_chol(nU, bw, B);
  if (st == 0) orc_band_solve(nU, bw, B, 1, u);
  free(B);
  return st == 0 ? ORC_OK : ORC_ENOTSPD;
}

/* ------------------------------------------------------------------------ */
/* Local matrices for the reduced-basis oracle (dense, small m only).        */
/* ------------------------------------------------------------------------ */

/* K_II (dense nI x nI) and the Dirichlet lifts rhs^l = -K_IB g^l (4 x nI) for
 * one coarse element.  Either output may be NULL. */
int orc_cell_system_dense(int m, const double* a, ptrdiff_t lda, int bc, double* KII, double* lift) {
  ensure_kref();
  const int nn = m + 1, ni = m - 1, nI = ni * ni;
  double* g = (double*)malloc(sizeof(double) * 4 * (size_t)nn * nn);
  if (!g) return ORC_ENOMEM;
  cell_boundary_data(m, a, lda, bc, g);
  if (KII) memset(KII, 0, sizeof(double) * (size_t)nI * nI);
  if (lift) memset(lift, 0, sizeof(double) * 4 * (size_t)nI);
  for (int ey = 0; ey < m; ++ey)
    for (int ex = 0; ex < m; ++ex) {
      double ae = a[(ptrdiff_t)ey * lda + ex];
      int px[4] = {ex, ex + 1, ex + 1, ex};
      int py[4] = {ey, ey, ey + 1, ey + 1};
      for (int al = 0; al < 4; ++al) {
        int ia = (px[al] > 0 && px[al] < m && py[al] > 0 && py[al] < m) ? (py[al] - 1) * ni + (px[al] - 1) : -1;
        if (ia < 0) continue;
        for (int be = 0; be < 4; ++be) {
          double kab = ae * KREF[4 * al + be];
          int ib = (px[be] > 0 && px[be] < m && py[be] > 0 && py[be] < m) ? (py[be] - 1) * ni + (px[be] - 1) : -1;
          if (ib >= 0) {
            if (KII) KII[(size_t)ia * nI + ib] += kab;
          } else if (lift) {
            int nid = py[be] * nn + px[be];
            for (int l = 0; l < 4; ++l) lift[(size_t)l * nI + ia] -= kab * g[(size_t)l * nn * nn + nid];
          }
        }
      }
    }
  free(g);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Synthetic coefficient: (base + amp sin(2 pi x/eps) sin(2 pi y/eps))       */
/*   * exp(beta * sum_j xi_j psi_j(x)),  psi_j(x) = (1 - |x-c_j|^2/rho^2)^2_+, */
/* with bump centres on a g x g cell-centred grid, j row-major.  Sampled at   */
/* fine-element centroids of the n x n fine grid on [0,1]^2.                  */
/* ------------------------------------------------------------------------ */

int orc_coef_bumps(int64_t N, int nfine, const double* xi, int nxi, int g, double rho, double eps, double base,
                   double amp, double beta, double* a, int nthreads) {
  if (N < 0 || nfine < 1 || g < 1 || nxi < g * g || !xi || !a) return ORC_EINVAL;
  const double h = 1.0 / nfine;
  const double pi = 3.14159265358979323846;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
  for (int64_t t = 0; t < N * nfine; ++t) {
    int64_t s = t / nfine;
    int iy = (int)(t % nfine);
    const double* xs = xi + s * nxi;
    for (int ix = 0; ix < nfine; ++ix) {
      double x = (ix + 0.5) * h, y = (iy + 0.5) * h;
      double field = 0.0;
      for (int j = 0; j < g * g; ++j) {
        double cx = ((j % g) + 0.5) / g, cy = ((j / g) + 0.5) / g;
        double r2 = ((x - cx) * (x - cx) + (y - cy) * (y - cy)) / (rho * rho);
        if (r2 < 1.0) field += xs[j] * (1.0 - r2) * (1.0 - r2);
      }
      double osc = base + amp * sin(2.0 * pi * x / eps) * sin(2.0 * pi * y / eps);
      a[(s * nfine + iy) * (int64_t)nfine + ix] = osc * exp(beta * field);
    }
  }
  return ORC_OK;
}

/* High-contrast channels-and-inclusions medium (synthetic stand-in for the
 * media of Sec. 5.1-5.2, which the paper gives only as figures).  Feature j
 * (kind 0: horizontal channel, 1: vertical channel, 2: square inclusion)
 * covers the fine elements (centroid xc, yc, cell size h = 1/nfine):
 *   horizontal: row floor(y0 nfine) and x0 <= xc <= x0 + size;
 *   vertical:   column floor(x0 nfine) and y0 <= yc <= y0 + size;
 *   square:     |xc - x0| <= size/2 and |yc - y0| <= size/2 (x0, y0 = centre).
 * a = theta_j of the highest-index feature covering the element, 1 where
 * none does, theta_j = 10^(decades * sigmoid(xi_j)) (the transform makes a
 * positive and bounded, Sec. 2.1.3). */
int orc_coef_features(int64_t N, int nfine, int nfeat, const int32_t* kind, const double* x0, const double* y0,
                      const double* size, const double* xi, int nxi, double decades, double* a, int nthreads) {
  if (N < 0 || nfine < 1 || nfeat < 0 || nxi < nfeat || !a || (N > 0 && !xi)) return ORC_EINVAL;
  const double h = 1.0 / nfine;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
  for (int64_t t = 0; t < N * nfine; ++t) {
    const int64_t s = t / nfine;
    const int iy = (int)(t % nfine);
    const double* xs = xi + s * nxi;
    for (int ix = 0; ix < nfine; ++ix) {
      const double xc = (ix + 0.5) * h, yc = (iy + 0.5) * h;
      double v = 1.0;
      for (int j = 0; j < nfeat; ++j) {
        int cover = 0;
        if (kind[j] == 0) {
          int row = (int)floor(y0[j] * nfine);
          if (row > nfine - 1) row = nfine - 1;
          cover = iy == row && xc >= x0[j] && xc <= x0[j] + size[j];
        } else if (kind[j] == 1) {
          int col = (int)floor(x0[j] * nfine);
          if (col > nfine - 1) col = nfine - 1;
          cover = ix == col && yc >= y0[j] && yc <= y0[j] + size[j];
        } else {
          cover = fabs(xc - x0[j]) <= 0.5 * size[j] && fabs(yc - y0[j]) <= 0.5 * size[j];
        }
        if (cover) v = pow(10.0, decades / (1.0 + exp(-xs[j])));
      }
      a[(s * nfine + iy) * (int64_t)nfine + ix] = v;
    }
  }
  return ORC_OK;
}
