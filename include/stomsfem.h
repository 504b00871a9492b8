/*
 * stomsfem.h -- C ABI of the MI355X (gfx950) implementation of the simultaneous
 * local upscaling step of the stochastic multiscale FEM of Hou, Li & Zhang,
 * "Exploring the locally low dimensional structure in solving random elliptic
 * PDEs" (StoMsFEM).
 *
 * Problem (Sec. 1, eq. eqn): -div(a(x,xi) grad u) = f on D = [0,1]^2, u = 0
 * on the boundary, for many samples xi.  D is cut into ncx x ncy square coarse
 * elements K (Sec. 2.2), each resolved by an m x m fine Q1 grid (m = H/h).
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers owned by the caller; they must
 *    stay valid until the work queued on `stream` has completed.  `stream` is
 *    a hipStream_t (NULL = the default stream).  Every call is asynchronous
 *    with respect to the host unless stated otherwise.
 *  - Coefficient samples a are piecewise constant per fine element (sampled at
 *    the element centroid), row-major [nsamples][ncy*m][ncx*m] (y index
 *    outer).  a_dtype selects float64 (STOMSFEM_F64) or float32 (STOMSFEM_F32).
 *  - Coarse element K = (kx, ky) has index ky*ncx + kx.  Its four nodes are
 *    numbered counter-clockwise from the lower-left corner: 0=(x0,y0),
 *    1=(x1,y0), 2=(x1,y1), 3=(x0,y1).  A 4x4 symmetric upscaled stiffness is
 *    stored as its 10 unique entries in the order 00,01,02,03,11,12,13,22,23,33.
 *  - Coarse unknowns are the interior coarse nodes (zero Dirichlet data) in
 *    natural order: node (ix, iy), 1 <= ix < ncx, 1 <= iy < ncy, has index
 *    (iy-1)*(ncx-1) + (ix-1).
 *  - Return value: STOMSFEM_OK or a negative stomsfem_status.  Argument errors
 *    are detected on the host before anything is queued.  Numerical events
 *    that concern one (element, sample) pair are reported in the optional
 *    per-pair `status` array and do not fail the call.  A failed HIP launch
 *    returns STOMSFEM_EHIP; faults inside kernels surface at the caller's next
 *    synchronising call.  stomsfem_last_error() gives a thread-local message.
 *  - Calls never print and never abort the process.
 *  - Ordering of shared scratch memory.  Entry points that use the
 *    library-owned workspace of a device (the coarse solves, the fine solve,
 *    the refined FP32 upscaling, the collocation quadrature) order themselves:
 *    each makes its stream wait for the previous such call's work (an event
 *    recorded on that call's stream) before queueing its own, so calls on
 *    different streams never use the workspace at the same time.  The same
 *    holds for the scratch buffers of one model (fallback lists and chunk
 *    buffers): every call that takes a model orders itself after the
 *    previous call on that model.  Streams under graph capture skip this
 *    ordering; graphs that capture such calls on several streams must order
 *    them themselves.
 */
#ifndef STOMSFEM_H
#define STOMSFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STOMSFEM_OK = 0,
  STOMSFEM_EINVAL = -1,   /* bad argument (caught on the host, nothing queued) */
  STOMSFEM_ENOMEM = -2,   /* device workspace could not be allocated */
  STOMSFEM_EHIP = -3,     /* a HIP runtime call or kernel launch failed */
  STOMSFEM_ENOTSPD = -4,  /* per pair: a pivot of the local/coarse factorisation was <= 0 or NaN */
  STOMSFEM_ENOCONV = -5,  /* per pair: mixed-precision refinement did not converge (result recomputed in FP64) */
  STOMSFEM_EVERSION = -6  /* model file / ABI version mismatch */
} stomsfem_status;

enum { STOMSFEM_F64 = 0, STOMSFEM_F32 = 1 };

/* Arithmetic of the local cell solves. */
enum {
  STOMSFEM_PREC_F64 = 0,           /* FP64 factorisation and energies */
  STOMSFEM_PREC_F32_REFINE64 = 1,  /* FP32 arithmetic where the entry point allows it, FP64 residuals/energies */
  STOMSFEM_PREC_BF16 = 2,          /* BF16 matrix-core products with FP32 accumulation (surrogate) */
  STOMSFEM_PREC_AUTO = 3,          /* stomsfem_upscale: the autotuner's choice for (m, a_dtype), else FP64 */
  STOMSFEM_PREC_F32 = 4,           /* plain FP32 arithmetic, no refinement: the reduced basis's matrix-core
                                      stage and the surrogate's FP32 reference */
  STOMSFEM_PREC_F16 = 5            /* FP16 matrix-core products (single terms) with FP32 accumulation
                                      (surrogate) */
};

/* Boundary data of the cell problems (Sec. 2.2 eq. MsFEB): linear (the
 * bilinear nodal functions on the boundary of K), or oscillatory (named for
 * Sec. 5.3 without a definition; here on each edge of K the 1-D discrete
 * harmonic profile of the edge-adjacent fine elements, sum_{s>=t} 1/a_s /
 * sum_s 1/a_s from the edge's first corner, which is exact for media layered
 * across the edge and equals the linear data for a constant coefficient). */
enum { STOMSFEM_BC_LINEAR = 0, STOMSFEM_BC_OSCILLATORY = 1 };

#define STOMSFEM_ABI_VERSION 1

/* ABI version (STOMSFEM_ABI_VERSION of the built library). */
int stomsfem_version(void);

/* Human-readable description of the last error on the calling thread. */
const char* stomsfem_last_error(void);

/* ------------------------------------------------------------------------
 * Coefficient samples of the synthetic bump family (the nonlinear transform
 * of Sec. 2.1.3, eq. nonlinear1, applied to an affine sum of local modes):
 *
 *   a(x, xi) = (base + amp sin(2 pi x1/eps) sin(2 pi x2/eps))
 *              * exp(beta * sum_j xi_j psi_j(x)),
 *   psi_j(x) = (1 - |x - c_j|^2 / rho^2)^2 for |x - c_j| < rho, else 0,
 *
 * with the g*g bump centres c_j = ((j mod g) + 1/2, floor(j/g) + 1/2) / g.
 * Sampled at the centroids of an nfine x nfine grid on [0,1]^2.
 *   xi : device [nsamples][nxi] float64, nxi >= g*g (only the first g*g used)
 *   a  : device out [nsamples][nfine][nfine] in a_dtype
 * ------------------------------------------------------------------------ */
int stomsfem_coef_bumps(int64_t nsamples, int32_t nfine, const double* xi, int32_t nxi, int32_t g, double rho,
                        double eps, double base, double amp, double beta, void* a, int32_t a_dtype,
                        void* stream);

/* ------------------------------------------------------------------------
 * High-contrast channels-and-inclusions medium (synthetic stand-in for the
 * media of Secs. 5.1-5.2, which exist only as figures): background 1 plus
 * nfeat features j (kind 0 = horizontal channel on fine row floor(y0*nfine),
 * covering centroids x0 <= xc <= x0 + size; kind 1 = vertical channel on
 * column floor(x0*nfine), y0 <= yc <= y0 + size; kind 2 = square of side
 * size centred at (x0, y0), |xc - x0| <= size/2 and |yc - y0| <= size/2).
 * A fine element takes the conductivity of the highest-index feature that
 * covers it,  theta_j = 10^(decades / (1 + exp(-xi_j)))  (a bounded positive
 * transform of a Gaussian variable, Sec. 2.1.3).
 *
 * stomsfem_feature_map: map device int32 [nfine][nfine] = that index or -1;
 *   kind, x0, y0, size device arrays [nfeat], nfeat <= 1024.  Asynchronous.
 * stomsfem_coef_features: a device [nsamples][nfine][nfine] (a_dtype) from
 *   the map and xi device [nsamples][nxi] (nxi >= nfeat).  Asynchronous.
 * ------------------------------------------------------------------------ */
int stomsfem_feature_map(int32_t nfine, int32_t nfeat, const int32_t* kind, const double* x0, const double* y0,
                         const double* size, int32_t* map, void* stream);
int stomsfem_coef_features(int64_t nsamples, int32_t nfine, const int32_t* map, int32_t nfeat, const double* xi,
                           int32_t nxi, double decades, void* a, int32_t a_dtype, void* stream);

/* ------------------------------------------------------------------------
 * Simultaneous local upscaling (Sec. 2.2 eqs. MsFEB and stiffness_local;
 * Sec. 3 eq. MsFEB2): for every coarse element K and every sample, solve the
 * cell problems -div(a grad phi^l) = 0 in K, phi^l = p^l on the boundary of
 * K, on the m x m fine Q1 grid, and form
 *
 *   S_ll' = int_K a grad phi^l . grad phi^l'      (l, l' = 0..3).
 *
 * One homogeneous batch shares ncx, ncy and m.  Several batches (for example
 * different m) are processed by one call.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t ncx, ncy;   /* coarse elements per direction (>= 1) */
  int32_t m;          /* fine cells per coarse element per direction (1..48) */
  int32_t a_dtype;    /* STOMSFEM_F64 or STOMSFEM_F32 */
  int64_t nsamples;   /* >= 0 */
  const void* a;      /* device [nsamples][ncy*m][ncx*m] */
  double* S;          /* device out [nsamples][ncy*ncx][10] */
  int32_t* status;    /* device out [nsamples][ncy*ncx] per-pair status, or NULL */
} stomsfem_batch;

/*   batches   : host array of nbatch descriptors (read during the call only)
 *   precision : STOMSFEM_PREC_F64 -- FP64 factorisation (asynchronous);
 *               STOMSFEM_PREC_AUTO -- per batch, the precision the autotuner
 *               chose for its (m, a_dtype) (FP64 when untuned);
 *               STOMSFEM_PREC_F32_REFINE64 (m <= 32) -- FP32 band LDL^T of
 *               K_II, FP64 residuals r = f - K_II x with FP64 coefficients,
 *               x += (LDL^T)^{-1} r until max_l |r^l|_inf / |f^l|_inf <=
 *               STOMSFEM_REFINE_TOL (at most STOMSFEM_REFINE_MAXIT solves),
 *               S from the FP64 energy sum of the refined phi^l; pairs that
 *               do not converge are recomputed by the FP64 kernels.  Needs
 *               (m-1)^2 (4 m + 40) bytes of LDS per workgroup (161 KB at
 *               m = 32; EINVAL if the device allows less), uses the library
 *               workspace and synchronises `stream` once per batch.
 *   bc        : STOMSFEM_BC_LINEAR, or STOMSFEM_BC_OSCILLATORY (any m <= 48,
 *               FP64 only: served by the reference kernel, one workgroup per
 *               pair, so much slower than the linear data's tuned kernels;
 *               EINVAL with precision F32_REFINE64)
 * Per-pair status: STOMSFEM_OK; 1 = recomputed in FP64 because the
 * refinement did not converge (F32_REFINE64 only); STOMSFEM_ENOTSPD when a
 * pivot of the FP64 factorisation is not positive (a <= 0 or NaN somewhere
 * in K), S is then undefined for that pair. */
#define STOMSFEM_REFINE_TOL 1e-10
#define STOMSFEM_REFINE_MAXIT 8
int stomsfem_upscale(const stomsfem_batch* batches, int32_t nbatch, int32_t precision, int32_t bc, void* stream);

/* Same computation through the simple reference kernel (one workgroup per
 * pair, band window in LDS, any m); used to cross-check the tuned kernels.
 * bc: STOMSFEM_BC_LINEAR or STOMSFEM_BC_OSCILLATORY. */
int stomsfem_upscale_reference(const stomsfem_batch* batch, int32_t bc, void* stream);

/* The same computation as stomsfem_upscale (FP64 factorisation, linear
 * boundary data) for batches of different m in ONE persistent launch: a
 * single queue of work items spans all batches and every wavefront takes
 * items with an atomic counter until the queue is empty.  An item is one
 * wavefront's tile (6 pairs for m = 16 and 32, 64 pairs for m = 8); items are
 * taken in decreasing order of cost (all m = 32 items, then m = 16, then
 * m = 8), so the launch ends on the cheapest ones.  S and the per-pair status
 * are bitwise those of stomsfem_upscale.
 *   batches : host array of nbatch (1..8) descriptors, every m in {8, 16, 32}
 *             (EINVAL otherwise), all with the same a_dtype
 * Uses 8 bytes of the library-owned device workspace (ordered against the
 * other workspace users, see above); asynchronous. */
int stomsfem_upscale_queue(const stomsfem_batch* batches, int32_t nbatch, void* stream);

/* ------------------------------------------------------------------------
 * Batched coarse solve and quantity of interest (Sec. 2.2 eq. upscaleSUF;
 * Petrov-Galerkin load of eq. stiffness_local_petrov; Monte Carlo estimators
 * of Sec. 4.1.1).  For every sample: assemble the global coarse stiffness
 * from S[s][K], drop the boundary nodes (zero Dirichlet data), solve
 * S U = b in FP64, then
 *   qoi_mean[i] = (1/N) sum_s U[s][i],
 *   qoi_var[i]  = (1/N) sum_s U[s][i]^2 - qoi_mean[i]^2   (paper's estimator).
 *   S       : device [nsamples][ncy*ncx][10] float64
 *   load    : device [ncy*ncx][4] element loads b^K_l, or NULL for f = 1 with
 *             b^K_l = int_K p^l = H^2/4, H = 1/ncx (square elements)
 *   U       : device out [nsamples][(ncx-1)*(ncy-1)]
 *   qoi_mean, qoi_var : device out [(ncx-1)*(ncy-1)], each may be NULL
 *   status  : device out [nsamples] (OK or ENOTSPD), may be NULL
 * Uses library-owned device workspace (see stomsfem_workspace_reserve).
 * ------------------------------------------------------------------------ */
/* Element loads of a bilinear source for the `load` argument of the coarse
 * solves: b^K_l = int_K b p^l (the Petrov-Galerkin load of eq.
 * stiffness_local_petrov with the coarse bilinear test functions) for
 *   b(x, y) = f[0] + f[1] x + f[2] y + f[3] x y
 * (Sec. 5.3 takes b = 2 + x1 x2, i.e. f = {2, 0, 0, 1}), square elements of
 * side H = 1/ncx, element ky*ncx + kx = [kx H, (kx+1) H] x [ky H, (ky+1) H].
 *   f    : host array of 4 finite coefficients (read during the call)
 *   load : device out [ncy*ncx][4], local nodes counter-clockwise from the
 *          lower-left corner
 * Exact (2 x 2 Gauss rule on bilinear x bilinear).  Asynchronous. */
int stomsfem_element_loads(int32_t ncx, int32_t ncy, const double* f, double* load, void* stream);

int stomsfem_coarse_solve(int32_t ncx, int32_t ncy, int64_t nsamples, const double* S, const double* load,
                          double* U, double* qoi_mean, double* qoi_var, int32_t* status, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve, arguments and outputs as stomsfem_coarse_solve, with its factor
 * workspace and QoI partial sums in a fixed 64 MiB array of device memory
 * that the library holds on every GPU it runs on, from module load until the
 * process ends.  Samples are solved in chunks that fit that array, so any
 * nsamples works; a mesh whose single sample needs more than 64 MiB
 * ((ncx-1)(ncy-1)(ncx+1)+1 doubles) is rejected with EINVAL.  U and status
 * are bit-identical to stomsfem_coarse_solve's; qoi_mean and qoi_var may
 * differ in the last bits (the partial sums are grouped differently when the
 * array is smaller than the default workspace).  Calls no allocating
 * routine.  All calls on one GPU share the array and keep no state in it
 * between calls: calls that overlap on one GPU (on different streams, or
 * from different threads) race and give undefined results, so serialise
 * them.  Asynchronous on `stream`. */
int stomsfem_coarse_solve_noalloc(int32_t ncx, int32_t ncy, int64_t nsamples, const double* S, const double* load,
                                  double* U, double* qoi_mean, double* qoi_var, int32_t* status, void* stream);

/* ------------------------------------------------------------------------
 * Oversampling with the Petrov-Galerkin local stiffness (Sec. 2.2: remark on
 * oversampling, eq. stiffness_local_petrov; Sec. 4.1.1 for the coarse solve).
 *
 * stomsfem_upscale_os: for every pair of `batch` the cell problems of
 * eq. MsFEB are solved on the patch of M = m + 2*oversample fine cells per
 * side centred on K (moved inside the domain where it would stick out), with
 * the bilinear nodal functions of the patch corners as boundary data; the
 * basis is recombined to take the nodal values delta_ik at the corners of K,
 * and
 *   S[l][l'] = int_K a grad phi^l . grad p^l'   (p^l': K's bilinear functions)
 * is written as 16 row-major doubles per pair (l: trial, l': test; corners
 * counter-clockwise from the lower left) to batch->S, which must therefore
 * hold [nsamples][ncy*ncx][16].  S is not symmetric when oversample > 0;
 * oversample = 0 gives the unpacked stiffness of stomsfem_upscale.  The
 * oversampling ratio is M/m (2 for oversample = m/2).  Requires
 * 2 <= M <= 64 and M <= ncx*m, ncy*m (EINVAL otherwise); patches of 16,
 * 20, 24, 25, 28, 30, 35, 36, 42, 45, 49, 50, 54, 60, 63 and 32 to 64 cells
 * in steps of 8 take the register-tiled kernel, others
 * one wavefront per pair with the band window in LDS.  Per-pair status
 * ENOTSPD if a pivot is not positive or the corner values of the patch
 * solutions are singular (S undefined).  Asynchronous.
 *
 * stomsfem_coarse_solve_pg: the coarse solve of stomsfem_coarse_solve for
 * the non-symmetric system assembled from S16 [nsamples][ncy*ncx][16]: the
 * equation of interior test node a is sum_b G[a][b] U_b = b_a with
 * G[a][b] = sum_K S^K[l(b)][l'(a)] (l(b), l'(a): the nodes' local indices in
 * K); FP64 LU without pivoting.  Same arguments, outputs and workspace use
 * as stomsfem_coarse_solve; requires ncx <= 64; status ENOTSPD if a pivot is
 * not positive.
 * ------------------------------------------------------------------------ */
int stomsfem_upscale_os(const stomsfem_batch* batch, int32_t oversample, void* stream);
int stomsfem_coarse_solve_pg(int32_t ncx, int32_t ncy, int64_t nsamples, const double* S16, const double* load,
                             double* U, double* qoi_mean, double* qoi_var, int32_t* status, void* stream);

/* ------------------------------------------------------------------------
 * The short-correlation Gaussian medium of Sec. 5.3 (eqs. mediaEx2,
 * betaCov) and its local KL parametrization on the coarse elements (Sec. 2.1,
 * eqs. domainpar, localKL, local_KL_truncation).
 *
 * stomsfem_coef_gauss: kappa = 0.1 + exp(beta) at the element centroids of
 * the nfine x nfine grid, beta(x) = sqrt(2/J) sum_j cos(w_j . x + phi_j)
 * (randomized spectral method for the covariance
 * exp(-dx^2/l1^2 - dy^2/l2^2)) with w_j = sqrt(2) (z[s][j][0]/l1,
 * z[s][j][1]/l2) and phi_j = 2 pi u[s][j]; z device [nsamples][J][2]
 * (standard normals), u device [nsamples][J] (uniform on [0, 1)), 1 <= J =
 * nterms <= 1024.  kappa device [nsamples][nfine][nfine]; beta (same shape)
 * may be NULL.  Asynchronous.
 *
 * stomsfem_local_kl (host only, needs no GPU): the K (<= 16) leading
 * eigenpairs of the covariance of beta between the m x m element centroids
 * (spacing h) of one coarse element: mu (host [K], descending) and unit
 * modes (host [K][m][m], row = y), from the separable structure (products
 * of the eigenpairs of the two one-dimensional m x m covariance matrices);
 * the discrete KL is beta ~ sum_k sqrt(mu_k) xi_k modes_k with
 * xi_k = modes_k . beta / sqrt(mu_k).  captured (host, may be NULL) = the
 * kept fraction of the trace.  Mode signs are arbitrary.
 *
 * stomsfem_kl_project: xi device [nsamples][nc*nc][K] of every (sample,
 * coarse element) from beta device [nsamples][nc m][nc m] with mu, modes
 * (device copies of the local_kl outputs); outside device [nsamples][nc*nc]
 * (may be NULL) = 1 where some |xi_k| > box; count (device uint64, may be
 * NULL) receives the number of such pairs (cleared first).  Asynchronous.
 *
 * stomsfem_kl_project_patches: the same on the oversampled patches of
 * Sec. 2.2, the domains on which Sec. 5.3 takes the local KL: the patch of
 * coarse element (kx, ky) is the element widened by `oversample` fine cells
 * on each side, moved inside the domain where it would stick out (first
 * cell along an axis: min(max(k m - oversample, 0), nc m - (m + 2
 * oversample))), so every patch has side m + 2 oversample and modes device
 * [K][m + 2 oversample][m + 2 oversample] (local_kl with that side) serve
 * all of them.  oversample = 0 is stomsfem_kl_project.  EINVAL if
 * oversample < 0 or the patch is wider than the domain.
 *
 * stomsfem_kl_blocks: the truncated coefficient 0.1 + exp(sum_{k < Kuse}
 * sqrt(mu_k) xi_k modes_k) on every pair's element, blocks device
 * [npairs][m][m], from xi device [npairs][K]; the blocks are a batch of
 * 1 x 1 meshes for stomsfem_upscale.  Asynchronous.
 * ------------------------------------------------------------------------ */
int stomsfem_coef_gauss(int64_t nsamples, int32_t nfine, int32_t nterms, const double* z, const double* u, double l1,
                        double l2, double* beta, double* kappa, void* stream);
int stomsfem_local_kl(int32_t m, double h, double l1, double l2, int32_t K, double* mu, double* modes,
                      double* captured);
int stomsfem_kl_project(int64_t nsamples, int32_t nc, int32_t m, const double* beta, int32_t K, const double* mu,
                        const double* modes, double box, double* xi, int32_t* outside, uint64_t* count,
                        void* stream);
int stomsfem_kl_project_patches(int64_t nsamples, int32_t nc, int32_t m, int32_t oversample, const double* beta,
                                int32_t K, const double* mu, const double* modes, double box, double* xi,
                                int32_t* outside, uint64_t* count, void* stream);
int stomsfem_kl_blocks(int64_t npairs, int32_t m, int32_t Kuse, int32_t K, const double* xi, const double* mu,
                       const double* modes, double* blocks, void* stream);


/* ------------------------------------------------------------------------
 * Fine-grid FEM and the two-level Monte Carlo estimator (Sec. 4.1.1, the
 * remark with eqs. MCmean2level and mseML).
 *
 * stomsfem_fine_solve: the global Q1 FEM on the nfine x nfine fine mesh of
 * [0,1]^2 (2 <= nfine <= 8192) with the piecewise-constant coefficient a
 * (device [nsamples][nfine][nfine], FP64, element row-major, y outer), f = 1
 * and zero Dirichlet data: u device [nsamples][(nfine-1)^2], interior fine
 * nodes in natural order.  For nfine <= 64 it is the coarse system of the
 * m = 1 upscaled elements (S = a_e K_Q1, load h^2/4 per element node), run
 * through the upscaling and banded coarse-solve kernels in chunks of samples
 * (status: ENOTSPD if a pivot is not positive, e.g. a <= 0); for larger
 * meshes it is stomsfem_fine_solve_pcg with tolerance
 * STOMSFEM_FINE_PCG_TOL and at most STOMSFEM_FINE_PCG_MAXIT iterations
 * (status: ENOCONV if not reached).  status device [nsamples] or NULL.  Uses
 * the library workspace; asynchronous on `stream` for nfine <= 64, otherwise
 * it synchronises `stream` every few iterations.
 *
 * stomsfem_fine_solve_pcg: the same system by conjugate gradients
 * preconditioned with one geometric multigrid V-cycle per iteration
 * (coefficients averaged over 2 x 2 elements per coarser level while the
 * element count per side is even and >= 8, bilinear interpolation and its
 * transpose, two damped-Jacobi sweeps before and after the coarse
 * correction, thirty on the coarsest level; FP64 throughout), for every
 * sample until ||b - K u||_2 <= tol ||b||_2 or max_iter iterations.  iters
 * device int32 [nsamples] or NULL: the iterations each sample took; status
 * device [nsamples] or NULL: OK or ENOCONV.  Samples in chunks of at most
 * 64 (about 65 MB each at nfine = 1024, in the library workspace).  Reads a
 * counter back every four iterations, so it synchronises `stream`.
 *
 * stomsfem_two_level_mc: per interior coarse node i of the nc x nc mesh,
 * mean[i] = M[U_H][i] + M[u_h - U_Hh][i] over the two sample sets (U_H device
 * [n_H][(nc-1)^2]; U_Hh device [n_h][(nc-1)^2] and u_fine device
 * [n_h][(nc m-1)^2] of the same second set), u_h taken at the fine node
 * (px m, py m) of coarse node (px, py); var_H[i] and var_d[i] the sample
 * variances (1/N normalisation) of U_H and of u_h - U_Hh, from which the
 * sampling part of the MSE is H^2 sum_i (var_H/n_H + var_d/n_h).  Any output
 * may be NULL.  Fixed summation order.  Asynchronous on `stream`.
 * ------------------------------------------------------------------------ */
#define STOMSFEM_FINE_PCG_TOL 1e-12
#define STOMSFEM_FINE_PCG_MAXIT 500
int stomsfem_fine_solve(const double* a, int32_t nfine, int64_t nsamples, double* u, int32_t* status,
                        void* stream);
int stomsfem_fine_solve_pcg(const double* a, int32_t nfine, int64_t nsamples, double tol, int32_t max_iter,
                            double* u, int32_t* iters, int32_t* status, void* stream);
int stomsfem_two_level_mc(const double* U_H, int64_t n_H, const double* U_Hh, const double* u_fine, int64_t n_h,
                          int32_t nc, int32_t m, double* mean, double* var_H, double* var_d, void* stream);

/* ------------------------------------------------------------------------
 * Reduced-basis acceleration (Sec. 3.2: eqs. KLphi, localRB, localRBsystem,
 * RBaffine/localAF; Algorithms 3 and 4).
 *
 * stomsfem_reduce (offline, Algorithm 3): from the training coefficient
 * samples `train` (S and status are not used and may be NULL), solve the cell
 * problems for phi^l, l = 0..2, and per patch K form the mean phibar^l and
 * the KL expansion of the centred phi^l in the energy inner product of
 * K_II(abar) (abar = training mean of the coefficient), with one shared basis
 * for the three l.  r_K = min(r_max, smallest r whose relative tail
 * sqrt(sum_{q>r} lambda_q / sum lambda_q) <= tail_tol, number of eigenvalues
 * above 1e-12 lambda_max: the numerical rank of the snapshots, 0 for a
 * single training sample).  The model stores,
 * per patch and fine element e, the P = r(r+1)/2 + 3r + 6 coefficients that
 * make the online Galerkin system a linear function of the coefficient
 * values a_e (the Q1 stiffness is affine in a_e).  Requires 2 <= m <= 48,
 * 1 <= r_max <= 8 and min((m-1)^2, 3 ntrain) <= 1024 (the eigenproblem: with
 * fewer snapshots than interior unknowns, 3 ntrain < (m-1)^2, the modes come
 * from the 3 ntrain x 3 ntrain snapshot matrix in the energy inner product,
 * the method of snapshots).  The training phi are FP64 banded solves: the
 * band in LDS up to m = 26, beyond that the band-window kernel (band rows in
 * an LDS ring, the finished factor rows in a device row store of about
 * (m-1)^2 (m+4) doubles for each of up to 1024 pairs in flight).  Allocates device memory (owned by the model) and
 * synchronises `stream` before returning.
 *
 * stomsfem_reduce_apply (online, Algorithm 4): S_rb for every pair of
 * `batch` (same ncx, ncy, m as the training batch):
 *   [A, Fh, B] = a_K^T G_K,   S_ll' = B_ll' - Fh_l . A^{-1} Fh_l'
 * precision STOMSFEM_PREC_F32 (the default online stage):
 * FP32 MFMA GEMM with FP32 accumulation, FP32 r x r solve;
 * STOMSFEM_PREC_F64: FP64 throughout (reference).  Per-pair status ENOTSPD
 * if the r x r system is not positive definite.  Asynchronous.
 * ------------------------------------------------------------------------ */
typedef struct stomsfem_model stomsfem_model;

int stomsfem_reduce(const stomsfem_batch* train, int32_t r_max, double tail_tol, stomsfem_model** model,
                    void* stream);
int stomsfem_reduce_apply(const stomsfem_model* model, const stomsfem_batch* batch, int32_t precision,
                          void* stream);

/* ------------------------------------------------------------------------
 * Reduced basis on oversampled patches (Sec. 3.2 on the patches of the
 * oversampled Petrov-Galerkin MsFEM of Sec. 2.2; the high-contrast example
 * of Sec. 5.2 uses the two together).
 *
 * stomsfem_reduce_os (offline): the cell problems of element K are those of
 * stomsfem_upscale_os, posed on the patch of Mp = m + 2*oversample fine
 * cells per side around K (moved inside the domain where it would stick
 * out) with the bilinear data of the patch corners.  From the training
 * samples `train` (device [ntrain][ncy*m][ncx*m]; S and status unused, may
 * be NULL) the patch blocks are reduced exactly as the elements of
 * stomsfem_reduce: means phibar^l, KL modes of the centred patch solutions
 * in the energy inner product of the training-mean coefficient, r_K by the
 * same rule.  Requires 2 <= Mp <= 64, Mp <= ncx*m and ncy*m,
 * 1 <= r_max <= 8, 1 <= ntrain <= 341 and the eigenproblem limit of
 * stomsfem_reduce (EINVAL otherwise); patches of more than 32 cells take
 * their snapshots from a band-window kernel (one wavefront per pair, the
 * finished factor rows in a device row store of about (Mp-1)^2 (Mp+4)
 * doubles for each of up to 1024 pairs in flight).  Allocates device memory (owned by the
 * model; a gathered copy of the training patches, ntrain*M*Mp*Mp doubles,
 * only during the call) and synchronises `stream`.  model_export 0..3 return
 * the patch quantities ((Mp-1)^2 interior nodes); stomsfem_model_save /
 * _load keep the model (kind 9).
 *
 * stomsfem_reduce_os_apply (online): for every pair of `batch` (same ncx,
 * ncy, m as the training batch) the reduced patch solutions
 *   psi^l = phibar^l + sum_q c^l_q zeta_q,  A c^l = -Fh_l (l = 0..2),
 *   psi^3 = 1 - sum_l psi^l,
 * recombined as in stomsfem_upscale_os: Psi[k][j] = psi^j at K's corners
 * (counter-clockwise from the lower left), phi^i = sum_j (Psi^{-T})[i][j]
 * psi^j, and
 *   S[i][l'] = int_K a grad phi^i . grad p^l'   (p^l': K's bilinear functions)
 * written as 16 row-major doubles per pair to batch->S ([nsamples][ncy*ncx]
 * [16]).  precision STOMSFEM_PREC_F32: the linear quantities (A, Fh and
 * the element sums over K) by one FP32 matrix-core GEMM [128 samples x
 * Mp^2] x [Mp^2 x 112] per workgroup with FP32 accumulation, then the r x r
 * solve and the recombination in FP64 per pair; STOMSFEM_PREC_F64: FP64
 * throughout (reference).  Per-pair status ENOTSPD if the r x r system is
 * not positive definite or Psi is singular.  Asynchronous.
 * ------------------------------------------------------------------------ */
int stomsfem_reduce_os(const stomsfem_batch* train, int32_t oversample, int32_t r_max, double tail_tol,
                       stomsfem_model** model, void* stream);
int stomsfem_reduce_os_apply(const stomsfem_model* model, const stomsfem_batch* batch, int32_t precision,
                             void* stream);

/* Copy model data to host memory (synchronous).  which:
 *   0 = r per patch        (int32  [ncy*ncx])
 *   1 = eigenvalues lambda (double [ncy*ncx][(m-1)^2], descending)
 *   2 = modes Z            (double [ncy*ncx][(m-1)^2][8], columns >= r_K are 0)
 *   3 = means phibar       (double [ncy*ncx][3][(m-1)^2])
 * (reduced-basis models), and for interpolation models:
 *   4 = node table         (double [rows][10], rows = sum_K nnodes^k_K)
 *   5 = row offsets        (int64  [ncy*ncx + 1]; patch K owns rows
 *                           off[K] .. off[K+1]-1)
 * bytes must equal the size of the array. */
int stomsfem_model_export(const stomsfem_model* model, int32_t which, void* host_dst, int64_t bytes);

/* Free a model (synchronous with respect to the device). */
int stomsfem_model_free(stomsfem_model* model);

/* ------------------------------------------------------------------------
 * Learned surrogate.  A per-patch multilayer perceptron maps the patch's
 * local random variables (the xi_j whose mode touches K: the local
 * parametrization of Sec. 3, eq. MsFEB2, at most 4, zero padded) to the 10
 * unique entries of S_K: 4 -> 64 -> 64 -> 64 -> 2 x 10, GELU(z) = z Phi(z),
 * two output heads, targets standardised per patch and entry with the
 * training mean and standard deviation.  Parameters per patch
 * (STOMSFEM_MLP_NPARAM floats, row-major, in this order): W1[4][64], b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], W4[64][20], b4[20].
 * Gate per pair (tolerance tau): S = (S_A + S_B)/2 of the heads,
 *   residual    = max_l |sum_l' S_ll'| / max|S|,
 *   uncertainty = max|S_A - S_B| / max|S|,
 * accepted if both <= tau and every local variable lies in [-box, box];
 * accepted S are projected to zero row sums (S <- P S P, P = I - 1 1^T/4).
 * Rejected pairs, and 1% of accepted pairs chosen by a hash of the pair index
 * ((p * 2654435761) mod 100 == 0, p = s*M + K) for auditing, are recomputed
 * by the plain FP64 path with the coefficient regenerated from xi: a fused
 * kernel for m = 8 (asynchronous); for other m the listed pairs' coefficient
 * blocks go through the upscaling kernels in chunks, after one synchronous
 * read of their number.
 * ------------------------------------------------------------------------ */
#define STOMSFEM_MLP_NPARAM 9940
#define STOMSFEM_MLP_BATCH 32

typedef struct {
  int32_t g;                             /* g x g bumps */
  double rho, eps, base, amp, beta;      /* see stomsfem_coef_bumps */
} stomsfem_bump_family;

/* Local variables of every patch for the bump family (host computation):
 * local_vars[K][kmax] = the indices j (increasing) of the bumps whose support
 * contains a fine-element centroid of K, -1 padded; nlocal[K] their number
 * (may be NULL).  EINVAL if a patch has more than kmax. */
int stomsfem_local_vars_bumps(int32_t ncx, int32_t ncy, int32_t m, const stomsfem_bump_family* fam, int32_t kmax,
                              int32_t* local_vars, int32_t* nlocal);

/* Create a surrogate for the bump family (1 <= m <= 48): local_vars host [M][4], init_params host
 * [M][STOMSFEM_MLP_NPARAM] (the caller draws the initial weights), fam = the
 * coefficient family used by the fallback, box = training box of the local
 * variables.  Synchronous. */
int stomsfem_mlp_create(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars, const float* init_params,
                        const stomsfem_bump_family* fam, double box, stomsfem_model** model);

/* Training pairs from the plain path: xi device [ntrain][nxi], S device
 * [ntrain][M][10].  Computes the standardisation and the per-patch inputs
 * and targets (device copies owned by the model). */
int stomsfem_mlp_set_data(stomsfem_model* model, const double* xi, int32_t nxi, const double* S, int64_t ntrain,
                          void* stream);

/* Surrogate for the channels-and-inclusions medium (stomsfem_coef_features)
 * on an nc x nc coarse mesh (nfine = nc*m).  The local variables of K are
 * the features that cover a fine element of K (the local parametrization of
 * Sec. 3, eq. MsFEB2, for this medium); a patch with more than 4 always takes
 * the plain path.  The network sees 2/(1 + exp(-xi_j)) - 1 (the covered
 * fraction of the decades, in [-1, 1]) instead of xi_j and predicts S_K
 * divided by the mean conductivity over the fine elements along the boundary
 * of K (the linear boundary conditions prescribe the gradient there, so max|S_K|
 * follows this mean over the decades); the gate's residual and uncertainty are
 * ratios and do not change with that scale.  map device
 * [nfine][nfine] (stomsfem_feature_map), copied; decades as in
 * stomsfem_coef_features; init_params host [nc*nc][STOMSFEM_MLP_NPARAM];
 * box bounds the local variables (in xi).  The plain fallback regenerates the
 * listed pairs' coefficient blocks from the map for every m.  Such a model is
 * not saved by stomsfem_model_save (EINVAL).  Synchronous.
 * stomsfem_local_vars_features: the same local variables on the host from a
 * host map [ncy*m][ncx*m]: local_vars[K][kmax] increasing, -1 padded, or
 * {-2, -1, ..} when K has more than kmax; nlocal[K] their number (may be
 * NULL).  EINVAL for a map entry outside [-1, nfeat). */
int stomsfem_local_vars_features(int32_t ncx, int32_t ncy, int32_t m, const int32_t* map, int32_t nfeat,
                                 int32_t kmax, int32_t* local_vars, int32_t* nlocal);
int stomsfem_mlp_create_features(int32_t nc, int32_t m, const int32_t* map, int32_t nfeat, double decades,
                                 const float* init_params, double box, stomsfem_model** model);

/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on
 * minibatches of STOMSFEM_MLP_BATCH pairs per patch taken cyclically from
 * perm (device int64 [ntrain], NULL = identity order); FP32 forward and
 * backward on the GPU.  loss (device [M], may be NULL) receives the last
 * minibatch loss per patch. */
int stomsfem_mlp_train(stomsfem_model* model, int32_t steps, float lr, const int64_t* perm, float* loss, void* stream);

/* Gradient of the loss for one explicit minibatch (no update): xb device
 * [M][32][4], tb device [M][32][10] (standardised targets), grads device
 * [M][STOMSFEM_MLP_NPARAM], loss device [M] or NULL. */
int stomsfem_mlp_grad(const stomsfem_model* model, const float* xb, const float* tb, float* grads, float* loss,
                      void* stream);

/* Copy the parameters out to dst (any memory) and/or in from src (either may
 * be NULL); asynchronous on stream. */
int stomsfem_mlp_params(stomsfem_model* model, float* dst, const float* src, void* stream);

/* Standardisation of the targets (host [M][10] each; either may be NULL). */
int stomsfem_mlp_standardization(const stomsfem_model* model, double* mu_host, double* sd_host);

/* Raw network outputs Y device [nsamples][M][20] for xi device
 * [nsamples][nxi]; precision STOMSFEM_PREC_BF16 (matrix cores, three-term
 * bf16 splitting), STOMSFEM_PREC_F16 (matrix cores, single fp16 terms) or
 * STOMSFEM_PREC_F32 (FP32 reference). */
int stomsfem_mlp_predict(const stomsfem_model* model, const double* xi, int32_t nxi, int64_t nsamples, float* Y,
                         int32_t precision, void* stream);

/* The surrogate's gate (the residual/uncertainty gate that decides between
 * the network and the plain local solve; the counterpart of the out-of-range
 * fallback in the remark after Algorithm 2, Sec. 3.1) applied to given raw
 * network outputs, with the same device code the surrogate path runs after
 * its forward pass.  Y device float [nsamples][M][20]: two heads of the 10
 * standardised entries; xi device [nsamples][nxi], read only for the box test
 * of the patch's local variables.  Per pair, with S_A and S_B the
 * de-standardised heads and S = (S_A + S_B)/2:
 *   residual    = max_l |sum_l' S_ll'| / max|S|,
 *   uncertainty = max|S_A - S_B| / max|S|;
 * accepted iff all 20 de-standardised values are finite, max|S| > 0, both
 * signals are <= gate_tol and every local variable lies in the model's box.
 * Outputs: S device [nsamples][M][10] = P S P (P = I - 1 1^T/4) where
 * accepted, S elsewhere; status device int32 [nsamples][M] (0 accepted,
 * 1 rejected) or NULL; gate device [nsamples][M][2] (residual, uncertainty;
 * NaN when a de-standardised value is not finite) or NULL.  No audit and no
 * fallback solve.  Asynchronous. */
int stomsfem_mlp_gate(const stomsfem_model* model, const float* Y, const double* xi, int32_t nxi, int64_t nsamples,
                      double gate_tol, double* S, int32_t* status, double* gate, void* stream);

/* Surrogate upscaling with gate and plain fallback: S device
 * [nsamples][M][10]; status device [nsamples][M] or NULL: 0 = surrogate
 * accepted, 1 = recomputed by the plain path (gate), 2 = audited (plain),
 * STOMSFEM_ENOTSPD from a fallback solve.  stats device uint64[4] or NULL,
 * accumulated (not cleared): [0] gate rejections, [1] audits, [2] max relative
 * error max|S_pred - S|/max|S| of rejected predictions, [3] same for audited
 * accepted ones (as IEEE-754 double bit patterns).  May grow a model-owned
 * buffer (a synchronous allocation) when nsamples exceeds earlier calls. */
int stomsfem_upscale_surrogate(stomsfem_model* model, const double* xi, int32_t nxi, int64_t nsamples, double* S,
                               int32_t* status, double gate_tol, int32_t precision, uint64_t* stats, void* stream);

/* ------------------------------------------------------------------------
 * Random interpolation (Sec. 3.1, Algorithms 1 and 2; error in Sec. 3.1.1).
 *
 * stomsfem_interp_build (offline, Algorithm 1): for every patch K with k_K
 * local variables (local_vars host [M][4], increasing indices < g*g, -1
 * padded at the end, as from stomsfem_local_vars_bumps), the tensor grid of
 * nnodes (2..9) Chebyshev-Gauss-Lobatto points per variable on the box
 * [lo, hi],  t_d = lo + (cos(pi d / (nnodes-1)) + 1)(hi - lo)/2,  and S_K at
 * every node, computed on the GPU by the plain path (coefficients of the
 * bump family `fam` with the local variables at the node and every other
 * variable 0, which does not change a on K).  Row c of patch K holds the
 * node whose digit for local variable i is (c / nnodes^(k-1-i)) mod nnodes
 * (variable 0 slowest).  1 <= m <= 48.  Allocates device memory owned by the
 * model and synchronises `stream`.  ENOTSPD if a node's cell problem fails.
 *
 * stomsfem_interp_apply (online, Algorithm 2): S device [nsamples][M][10]
 * for xi device [nsamples][nxi]: the tensor Lagrange interpolant of every
 * entry at the pair's local variables, evaluated in FP64 in barycentric form.
 * Pairs with a local variable outside [lo, hi] (or NaN) are computed by the
 * plain path with the coefficient regenerated from xi (the remark after
 * Algorithm 2).  status device [nsamples][M] or NULL: 0 = interpolated,
 * 1 = computed plainly, STOMSFEM_ENOTSPD from such a solve.  *nfallback
 * (host, may be NULL) receives the number of plainly computed pairs.
 * Synchronises `stream` once (to read that number); may grow a model-owned
 * buffer (a synchronous allocation) when nsamples exceeds earlier calls.
 * ------------------------------------------------------------------------ */
int stomsfem_interp_build(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars,
                          const stomsfem_bump_family* fam, int32_t nnodes, double lo, double hi,
                          stomsfem_model** model, void* stream);
int stomsfem_interp_apply(stomsfem_model* model, const double* xi, int32_t nxi, int64_t nsamples, double* S,
                          int32_t* status, int64_t* nfallback, void* stream);

/* ------------------------------------------------------------------------
 * Sparse-grid stochastic collocation with search-and-plug-in dictionaries
 * (Sec. 4.1.2, global SC methods: eq. sparseintegration, the variance formula
 * after it, eqs. SCofflinecost and SConlinecost; the collocation
 * experiment of Sec. 5.2).  The random variables are independent and uniform on a box.
 *
 * stomsfem_sparse_grid (host only, needs no GPU): the Smolyak sparse grid
 * of level `level` (0..8) in `dim` variables built from the nested
 * Clenshaw-Curtis rules (level 1: the midpoint; level i >= 2: 2^(i-1) + 1
 * points cos(pi j / 2^(i-1)) with the classical Clenshaw-Curtis weights),
 * with weights for the uniform probability measure (they sum to 1; some
 * are negative).  Points are integer digits c in 0..D, D = 2^max(level, 1),
 * standing for the node value lo + (cos(pi c / D) + 1)(hi - lo)/2 of the box
 * [lo, hi]; rows are in lexicographic order of the digits.  *npoints always
 * receives the number of points; with digits and weights both NULL nothing
 * else is written, otherwise digits (host [npoints][dim], may be NULL) and
 * weights (host [npoints], may be NULL) are filled and capacity must be at
 * least *npoints.  EINVAL for bad sizes or more than 2e6 terms in the
 * combination formula (binom(dim + level, level)).
 *
 * stomsfem_sc_build (offline): for the collocation points digits (host
 * [npoints][g*g], level `level`, box [lo, hi]) and the patches' local
 * variables (local_vars host [M][4] as for stomsfem_interp_build), the
 * dictionary of every patch K: its distinct local points (the points'
 * digits at K's local variables) and S_K at each, computed on the GPU by the
 * plain path (bump family `fam`, local variables at their node values, every
 * other variable 0, which does not change a on K).  1 <= m <= 48.  The
 * model owns its device memory (stomsfem_model_free); it cannot be saved.
 * Synchronises `stream`.  ENOTSPD if a cell problem fails.
 *
 * stomsfem_sc_apply (online search and plug-in): S device [npoints][M][10]
 * for digits device [npoints][nxi] (nxi >= g*g, the same level): every
 * (point, patch) looks its local point up in the patch's dictionary by
 * bisection and copies the stored S_K.  status device [npoints][M] or NULL:
 * 0 = found, 1 = the local point is not in the dictionary (S set to NaN).
 * Asynchronous on `stream`.
 *
 * stomsfem_quadrature: the collocation estimates mean[i] = sum_p w_p U[p][i]
 * and var[i] = sum_p w_p U[p][i]^2 - mean[i]^2 for U device [npoints][nu]
 * and weights w device [npoints]; mean, var device [nu] (either may be
 * NULL).  Summation in a fixed order (bitwise reproducible).  Uses the
 * library workspace; asynchronous on `stream`.
 * ------------------------------------------------------------------------ */
int stomsfem_sparse_grid(int32_t dim, int32_t level, int64_t capacity, int64_t* npoints, int32_t* digits,
                         double* weights);
int stomsfem_sc_build(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars,
                      const stomsfem_bump_family* fam, int32_t level, double lo, double hi, const int32_t* digits,
                      int64_t npoints, stomsfem_model** model, void* stream);
int stomsfem_sc_apply(const stomsfem_model* model, const int32_t* digits, int32_t nxi, int64_t npoints, double* S,
                      int32_t* status, void* stream);
int stomsfem_quadrature(const double* U, const double* w, int64_t npoints, int32_t nu, double* mean, double* var,
                        void* stream);

/* ------------------------------------------------------------------------
 * Sparse-grid interpolation of the upscaled stiffness in the local variables
 * (Sec. 3.1 with the sparse node sets of Sec. 4.1.2 and Sec. 5.3).
 *
 * stomsfem_sgi_build (offline): for every patch K with k_K <= 4 local
 * variables (local_vars host [M][4] as for stomsfem_interp_build), S_K at the
 * nodes of the level-`level` (0..5) Smolyak Clenshaw-Curtis grid in k_K
 * variables on the box [lo, hi] (node values as for stomsfem_sparse_grid),
 * computed on the GPU by the plain path (bump family `fam`, every other
 * variable 0).  1 <= m <= 48.  The model owns its device memory; it cannot be
 * saved.  Synchronises `stream`.  ENOTSPD if a node's cell problem fails.
 *
 * stomsfem_sgi_apply (online): S device [nsamples][M][10] for xi device
 * [nsamples][nxi]: Smolyak's combination of tensor Lagrange interpolants on
 * the nested nodes, evaluated in FP64 at the pair's local variables; pairs
 * with a local variable outside [lo, hi] (or NaN) are computed by the plain
 * path from xi.  status device [nsamples][M] or NULL: 0 = interpolated,
 * 1 = computed plainly, STOMSFEM_ENOTSPD from such a solve.  *nfallback
 * (host, may be NULL) receives the number of plainly computed pairs.  At most
 * 65535 coarse elements.  Synchronises `stream` once; may grow a
 * model-owned buffer (a synchronous allocation).
 * ------------------------------------------------------------------------ */
int stomsfem_sgi_build(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars,
                       const stomsfem_bump_family* fam, int32_t level, double lo, double hi, stomsfem_model** model,
                       void* stream);
int stomsfem_sgi_apply(stomsfem_model* model, const double* xi, int32_t nxi, int64_t nsamples, double* S,
                       int32_t* status, int64_t* nfallback, void* stream);

/* Interpolation of S in the local KL parameters (Sec. 5.3 with Sec. 3.1).
 *
 * stomsfem_kl_interp_build (offline): one table for every coarse element of
 * the ncx x ncy mesh (the covariance is translation invariant, so all
 * elements share mu, modes: device copies of the stomsfem_local_kl outputs,
 * K <= 4): S at the nnodes^K (2 <= nnodes <= 9) tensor Chebyshev-Gauss-
 * Lobatto nodes of [-box, box]^K (node ordering as stomsfem_interp_build),
 * computed by the plain path on the truncated coefficient of each node.
 * Synchronises `stream`; the model owns its device memory.
 *
 * stomsfem_kl_interp_apply (online): S device [nsamples][M][10] for the
 * local parameters xi device [nsamples][M][K] (from stomsfem_kl_project): the
 * tensor Lagrange interpolant where every parameter lies in [-box, box];
 * elsewhere (or NaN) the plain path on the sample's own coefficient block
 * from kappa device [nsamples][ncy m][ncx m] (FP64).  status device
 * [nsamples][M] or NULL: 0 = interpolated, 1 = computed plainly, ENOTSPD from
 * such a solve; *nfallback (host, may be NULL) = the number of plainly
 * computed pairs.  Synchronises `stream` once; may grow a model-owned buffer.
 *
 * stomsfem_kl_interp_os_build (offline): the same for the oversampled
 * Petrov-Galerkin stiffness (Sec. 2.2) in the parameters of the oversampled
 * patches, the setting of Sec. 5.3: mu, modes of side m + 2 oversample (from
 * stomsfem_local_kl with that side), 1 <= oversample <= m, m + 2 oversample
 * <= 64, square mesh.  An element's patch is moved inside the domain at the
 * edge, so along each axis the element sits at offset 0, oversample or
 * 2 oversample in it (first, interior, last elements); one table of the 16
 * entries (row-major [trial][test], as stomsfem_upscale_os) per pair of
 * offsets, nine in all.  A node's entries are those of an element with that
 * offset whose patch coefficient is the node's truncated local KL, computed
 * by the oversampling kernels on 3 x 3-element meshes.  The model is kind 7;
 * stomsfem_kl_interp_apply then writes S device [nsamples][M][16], xi from
 * stomsfem_kl_project_patches, and computes the out-of-box pairs by the
 * oversampling kernels on the sample's own patch.  ENOTSPD if a node's cell
 * problem fails.
 *
 * stomsfem_kl_sgi_os_build (offline): the same tables at the nodes of the
 * level-`level` (0..5) Smolyak sparse grid with nested Clenshaw-Curtis
 * (Chebyshev-Lobatto) nodes in the K patch parameters on [-box, box]^K (node
 * set as stomsfem_sparse_grid; 401 nodes at level 4 and 1105 at level 5 for
 * K = 4, close to the node count of Sec. 5.3), evaluated online by Smolyak's
 * combination of tensor Lagrange interpolants (as stomsfem_sgi_apply).  The
 * model is kind 8 and is applied by stomsfem_kl_interp_apply exactly as
 * kind 7 (S device [nsamples][M][16], the same fallback).  At most 65535
 * coarse elements. */
int stomsfem_kl_interp_build(int32_t ncx, int32_t ncy, int32_t m, int32_t K, const double* mu, const double* modes,
                             int32_t nnodes, double box, stomsfem_model** model, void* stream);
int stomsfem_kl_interp_apply(stomsfem_model* model, const double* xi, const double* kappa, int64_t nsamples,
                             double* S, int32_t* status, int64_t* nfallback, void* stream);
int stomsfem_kl_interp_os_build(int32_t ncx, int32_t ncy, int32_t m, int32_t oversample, int32_t K,
                                const double* mu, const double* modes, int32_t nnodes, double box,
                                stomsfem_model** model, void* stream);
int stomsfem_kl_sgi_os_build(int32_t ncx, int32_t ncy, int32_t m, int32_t oversample, int32_t K, const double* mu,
                             const double* modes, int32_t level, double box, stomsfem_model** model, void* stream);

/* ------------------------------------------------------------------------
 * Execution plans.  A stage is one batch of samples taken through the whole
 * path: coefficient generation from xi, local upscaling (FP64), coarse
 * assembly and solve with the Petrov-Galerkin load for f = 1, and the Monte
 * Carlo mean and variance of U over the batch (Sec. 2.2 eqs. MsFEB,
 * stiffness_local, upscaleSUF; Sec. 4.1.1).  stomsfem_plan_create groups the
 * stages by (ncx, m), gives every group its own device buffers and stream,
 * and captures HIP graphs: one for the whole plan, whose group branches run
 * concurrently (stages of one group run in order), and one per stage.
 * Replays allocate and synchronise nothing; replays of one plan must not
 * overlap (the groups' buffers are reused).  U and status of a stage are
 * left in group buffers when the stage gives NULL (overwritten by the next
 * stage of the group).  Square coarse meshes, 2 <= ncx <= 64.
 * ------------------------------------------------------------------------ */
enum { STOMSFEM_FAMILY_BUMPS = 0, STOMSFEM_FAMILY_FEATURES = 1 };

typedef struct {
  int32_t ncx, ncy, m;
  int64_t nsamples;
  int32_t a_dtype;                  /* storage of the generated coefficient */
  int32_t family;                   /* STOMSFEM_FAMILY_* */
  stomsfem_bump_family bumps;       /* family BUMPS: see stomsfem_coef_bumps */
  const int32_t* feature_map;       /* family FEATURES: device [ncy*m][ncx*m] */
  int32_t nfeat;
  double decades;
  const double* xi;                 /* device [nsamples][nxi] */
  int32_t nxi;
  double* U;                        /* device out [nsamples][(ncx-1)(ncy-1)] or NULL */
  double* qoi_mean;                 /* device out [(ncx-1)(ncy-1)] or NULL */
  double* qoi_var;                  /* device out [(ncx-1)(ncy-1)] or NULL */
  int32_t* status;                  /* device out [nsamples][ncx*ncy] or NULL */
} stomsfem_stage;

typedef struct stomsfem_plan stomsfem_plan;

/* Synchronous (allocates, captures). */
int stomsfem_plan_create(const stomsfem_stage* stages, int32_t nstage, stomsfem_plan** plan);
/* Replay the whole plan (stage = -1) or one stage on `stream`; asynchronous. */
int stomsfem_plan_launch(stomsfem_plan* plan, int32_t stage, void* stream);
/* Synchronous. */
int stomsfem_plan_free(stomsfem_plan* plan);

/* ------------------------------------------------------------------------
 * Autotuner of the plain upscaling kernels.  For the batch's (m, a_dtype) on
 * the current device it times, with HIP events over `reps` launches after a
 * warm-up, every launch shape (workgroup size 64/128/256 of the per-lane
 * kernel for m <= 8; 1 or 2 wavefronts per workgroup of the tiled kernel for
 * m = 16, 32), keeps only shapes whose S equals the default shape's bit for
 * bit, then times FP64 against STOMSFEM_PREC_F32_REFINE64 on a prefix of
 * about 16384 pairs (the refined variant must agree to 1e-10 relative).  The
 * fastest choice is recorded for the process and used by every later
 * stomsfem_upscale (launch shape; precision when the caller passes
 * STOMSFEM_PREC_AUTO) and by plans created afterwards.  Synchronous;
 * overwrites batch->S (left holding the chosen configuration's result).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t m, a_dtype;
  int32_t lane_block;     /* chosen workgroup size (m <= 8) */
  int32_t tiled_waves;    /* chosen wavefronts per workgroup (m = 16, 32) */
  int32_t precision;      /* STOMSFEM_PREC_F64 or STOMSFEM_PREC_F32_REFINE64 */
  int32_t candidates;     /* launch shapes timed */
  double ms_default;      /* default shape, ms per launch */
  double ms_best;         /* chosen shape, ms per launch */
} stomsfem_tuning;

int stomsfem_autotune(const stomsfem_batch* batch, int32_t reps, stomsfem_tuning* out, void* stream);
/* Forget the choices made on the current device. */
int stomsfem_tuning_reset(void);

/* ------------------------------------------------------------------------
 * Model files, counters, training alias.
 *
 * stomsfem_model_save: writes a reduced-basis (also on oversampled patches),
 *   random-interpolation or learned-surrogate model to `path`: a header (magic "STOMSFEM",
 *   ABI version, kind, mesh, scalars, coefficient family) followed by the
 *   model's device arrays, each preceded by (index, element size, count).
 *   The surrogate's training data are not written (stomsfem_mlp_set_data
 *   again before further training); a surrogate of the channels medium is
 *   not written (EINVAL).  Synchronous.
 * stomsfem_model_load: reads such a file onto the current device; the loaded
 *   model's online results are bitwise those of the saved one.
 *   STOMSFEM_EVERSION for a file of another ABI version or no model file,
 *   EINVAL for a corrupt one.  Synchronous.
 * stomsfem_stats_get / _reset: process-wide counters of pairs through the
 *   refined FP32 path and their FP64 recomputations, random-interpolation
 *   pairs and their out-of-box plain solves, surrogate pairs and their plain
 *   recomputations (for m != 8; at m = 8 the counts stay on the device, see
 *   the `stats` argument of stomsfem_upscale_surrogate).
 * stomsfem_surrogate_train: the same as stomsfem_mlp_train.
 * ------------------------------------------------------------------------ */
typedef struct {
  uint64_t refine_pairs, refine_recomputed;
  uint64_t interp_pairs, interp_fallbacks;
  uint64_t surrogate_pairs, surrogate_recomputed;
} stomsfem_stats;

int stomsfem_model_save(const stomsfem_model* model, const char* path);
int stomsfem_model_load(const char* path, stomsfem_model** model);
/* kind: 1 = reduced basis, 2 = learned surrogate, 3 = random interpolation,
 * 4 = sparse-grid collocation dictionaries, 5 = sparse-grid interpolation,
 * 6 = interpolation in the local KL parameters; 7 = the same for the oversampled
 * Petrov-Galerkin stiffness; 8 = the latter on a sparse grid; 9 = reduced
 * basis on oversampled patches (m = the element side);
 * any output pointer may be NULL. */
int stomsfem_model_shape(const stomsfem_model* model, int32_t* kind, int32_t* ncx, int32_t* ncy, int32_t* m);
int stomsfem_stats_get(stomsfem_stats* out);
int stomsfem_stats_reset(void);
int stomsfem_surrogate_train(stomsfem_model* model, int32_t steps, float lr, const int64_t* perm, float* loss,
                             void* stream);

/* Grow the library-owned device workspace of the current device to at least
 * `bytes` (the coarse solve needs 8*(ncx-1)*(ncy-1)*(ncx+1) bytes per sample
 * in flight).  Calls made after a large enough reservation allocate nothing.
 * Synchronous.  Returns OK or ENOMEM. */
int stomsfem_workspace_reserve(int64_t bytes);

/* Release the workspace of the current device (synchronous). */
int stomsfem_workspace_release(void);

#ifdef __cplusplus
}
#endif
#endif /* STOMSFEM_H */
