// Host side of the C ABI declared in include/stomsfem.h: argument
// validation, the library-owned device workspace, and kernel dispatch.
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <cmath>
#include <functional>
#include <map>
#include <tuple>

#include "common.h"
#include "rb.h"
#include "mlp.h"
#include "ri.h"
#include "mixed.h"
#include "sc.h"

namespace stomsfem {
hipError_t launch_upscale_small(const UpArgs& args, int a_dtype, hipStream_t st, int block);
hipError_t launch_upscale_ref(const UpArgs& args, int a_dtype, hipStream_t st);
size_t upscale_ref_lds_bytes(int m);
hipError_t launch_upscale_tiled(const UpArgs& args, int a_dtype, hipStream_t st, int waves);
bool tiled_supports(int m);
hipError_t launch_upscale_queue(const UpArgs* batches, int nb, int a_dtype, unsigned long long* counter,
                                hipStream_t st);
bool queue_supports(int m);
int queue_max_batches();
hipError_t launch_element_loads(int ncx, int ncy, const double* f, double* load, hipStream_t st);
hipError_t launch_coarse(int ncx, int ncy, int64_t N, const double* S, const double* load, double* U, double* mean,
                         double* var, int32_t* status, double* work, hipStream_t st);
hipError_t launch_coarse_pg(int ncx, int ncy, int64_t N, const double* S16, const double* load, double* U,
                            double* mean, double* var, int32_t* status, double* work, hipStream_t st);
int64_t fine_pcg_doubles_per_sample(int nfine);
hipError_t launch_fine_pcg(const double* a, int n, int64_t N, double tol, int max_iter, double* u, int32_t* iters,
                           int32_t* status, double* work, hipStream_t st);
hipError_t launch_coarse_capped(int ncx, int ncy, int64_t N, const double* S, const double* load, double* U,
                                double* mean, double* var, int32_t* status, double* work, int64_t work_cap,
                                hipStream_t st);
// list != nullptr: only the batch's pairs list[i] (i < nlist), S and status compact at i
hipError_t launch_upscale_os(const UpArgs& up, int o, int a_dtype, hipStream_t st, const int64_t* list = nullptr,
                             int64_t nlist = 0);
hipError_t launch_gauss_field(int64_t nsamples, int nfine, int J, const double* z, const double* u, double l1,
                              double l2, double* beta, double* kappa, hipStream_t st);
void local_kl_modes(int m, double h, double l1, double l2, int K, double* mu, double* modes, double* captured);
hipError_t launch_kl_project(int64_t npairs, int nc, int m, int o, int K, const double* beta, const double* mu,
                             const double* modes, double box, double* xi, int32_t* outside,
                             unsigned long long* count, hipStream_t st);
hipError_t launch_kl_blocks(int64_t npairs, int m, int Kuse, int K, const double* xi, const double* mu,
                            const double* modes, double* blocks, hipStream_t st);
hipError_t launch_embed_patch(int64_t count, int m, int o, int cx, int cy, const double* blocks, double* fields,
                              hipStream_t st);
hipError_t launch_pick_class(int64_t count, int cx, int cy, const double* S9, const int32_t* st9, double* dst,
                             int32_t* dst_status, hipStream_t st);
hipError_t launch_two_level(const double* UH, int64_t nH, const double* UHh, const double* uf, int64_t nh, int nc,
                            int m, double* mean, double* var_H, double* var_d, hipStream_t st);
bool upscale_os_supports(int m, int o);
int64_t coarse_work_doubles(int ncx, int ncy, int64_t nsamples);
size_t coarse_lds_bytes(int ncx, bool pg);
hipError_t launch_coef_bumps(int64_t nsamples, int nfine, const double* xi, int nxi, int g, double rho, double eps,
                             double base, double amp, double beta, void* a, int a_dtype, hipStream_t st);
hipError_t launch_feature_map(int nfine, int nfeat, const int32_t* kind, const double* x0, const double* y0,
                              const double* size, int32_t* map, hipStream_t st);
hipError_t launch_coef_features(int64_t nsamples, int nfine, const int32_t* map, int nfeat, const double* xi, int nxi,
                                double decades, void* a, int a_dtype, hipStream_t st);
}  // namespace stomsfem

using namespace stomsfem;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return STOMSFEM_EHIP;
}

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
  std::mutex lease;              // held by the call that uses the workspace
  hipEvent_t done = nullptr;     // recorded on the last user's stream when its call ended
};
std::mutex g_ws_mutex;
std::unordered_map<int, Workspace> g_ws;

// Grows w to at least `bytes` (the caller holds w.lease).  Growth frees the
// old buffer after a device synchronisation and is a synchronous hipMalloc.
int workspace_grow(Workspace& w, size_t bytes) {
  if (w.bytes >= bytes) return STOMSFEM_OK;
  hipError_t e;
  if (w.ptr) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    hipFree(w.ptr);
    w.ptr = nullptr;
    w.bytes = 0;
  }
  e = hipMalloc(&w.ptr, bytes);
  if (e != hipSuccess) {
    w.ptr = nullptr;
    (void)hipGetLastError();
    return fail(STOMSFEM_ENOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
  }
  w.bytes = bytes;
  return STOMSFEM_OK;
}

Workspace* workspace_of_current_device(int* rc) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *rc = hip_fail(e, "hipGetDevice");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_ws_mutex);
  *rc = STOMSFEM_OK;
  return &g_ws[dev];  // nodes of an unordered_map never move
}

// Orders the calls that share one piece of scratch memory.  While an
// OrderedUse lives, no other call holds the same mutex; its stream first
// waits for the work queued by the previous holder (the event that holder
// recorded on its own stream), and it records that event on its stream when
// it ends.  Calls on different streams therefore use the memory one after the
// other on the device instead of at the same time.  A stream under graph
// capture skips the event (a captured graph orders its own work).
class OrderedUse {
 public:
  OrderedUse() = default;
  OrderedUse(const OrderedUse&) = delete;
  OrderedUse& operator=(const OrderedUse&) = delete;
  int begin(std::mutex& mu, hipEvent_t& ev, hipStream_t st) {
    lk_ = std::unique_lock<std::mutex>(mu);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
      (void)hipGetLastError();
      cs = hipStreamCaptureStatusNone;
    }
    if (cs != hipStreamCaptureStatusNone) return STOMSFEM_OK;
    hipError_t e = hipSuccess;
    if (!ev) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    else e = hipStreamWaitEvent(st, ev, 0);
    if (e != hipSuccess) {
      lk_.unlock();
      return hip_fail(e, "stream ordering of shared scratch memory");
    }
    ev_ = &ev;
    st_ = st;
    return STOMSFEM_OK;
  }
  ~OrderedUse() {
    if (ev_ && *ev_) (void)hipEventRecord(*ev_, st_);
  }

 private:
  std::unique_lock<std::mutex> lk_;
  hipEvent_t* ev_ = nullptr;
  hipStream_t st_ = nullptr;
};

// The library workspace of the current device for one call, ordered against
// every other call that uses it (OrderedUse).
class WorkspaceLease {
 public:
  int acquire(size_t bytes, hipStream_t st, void** out) {
    int rc = STOMSFEM_OK;
    Workspace* w = workspace_of_current_device(&rc);
    if (!w) return rc;
    rc = use_.begin(w->lease, w->done, st);
    if (rc != STOMSFEM_OK) return rc;
    rc = workspace_grow(*w, bytes);
    if (rc != STOMSFEM_OK) return rc;
    *out = w->ptr;
    return STOMSFEM_OK;
  }

 private:
  OrderedUse use_;
};

// True when p is device (or managed) memory visible to the current device.
bool device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
#if HIP_VERSION_MAJOR >= 6
  const auto t = attr.type;
#else
  const auto t = attr.memoryType;
#endif
  return t == hipMemoryTypeDevice || t == hipMemoryTypeManaged;
}

int check_batch(const stomsfem_batch& b, int idx) {
  const std::string w = "batch " + std::to_string(idx) + ": ";
  if (b.ncx < 1 || b.ncy < 1) return fail(STOMSFEM_EINVAL, w + "ncx and ncy must be >= 1");
  if (b.m < 1 || b.m > 48) return fail(STOMSFEM_EINVAL, w + "m must be in 1..48");
  if (b.a_dtype != STOMSFEM_F64 && b.a_dtype != STOMSFEM_F32) return fail(STOMSFEM_EINVAL, w + "bad a_dtype");
  if (b.nsamples < 0) return fail(STOMSFEM_EINVAL, w + "nsamples < 0");
  if ((int64_t)b.ncx * b.m > (1 << 20) || (int64_t)b.ncy * b.m > (1 << 20))
    return fail(STOMSFEM_EINVAL, w + "fine grid too large");
  if (b.nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(b.a)) return fail(STOMSFEM_EINVAL, w + "a is not a device pointer");
  if (!device_ptr(b.S)) return fail(STOMSFEM_EINVAL, w + "S is not a device pointer");
  if (b.status && !device_ptr(b.status)) return fail(STOMSFEM_EINVAL, w + "status is not a device pointer");
  return STOMSFEM_OK;
}

UpArgs to_args(const stomsfem_batch& b) {
  UpArgs a;
  a.nsamples = b.nsamples;
  a.ncx = b.ncx;
  a.ncy = b.ncy;
  a.m = b.m;
  a.npairs = b.nsamples * (int64_t)b.ncx * b.ncy;
  a.a = b.a;
  a.S = b.S;
  a.status = b.status;
  a.bc = STOMSFEM_BC_LINEAR;
  return a;
}

}  // namespace

namespace stomsfem {
void set_last_error(const std::string& msg) { g_last_error = msg; }

// process-wide counters reported by stomsfem_stats_get
std::atomic<uint64_t> g_refine_pairs{0}, g_refine_recomputed{0}, g_interp_pairs{0}, g_interp_fallbacks{0},
    g_surrogate_pairs{0}, g_surrogate_recomputed{0};

// Launch configuration of the plain upscaling kernels per (device, m,
// coefficient dtype), chosen by stomsfem_autotune (defaults otherwise).
struct LaunchCfg {
  int lane_block = 64;   // workgroup size of the per-lane kernel (m <= 8)
  int tiled_waves = 1;   // wavefronts per workgroup of the tiled kernel (m = 16, 32)
  int precision = STOMSFEM_PREC_F64;
  double ms_default = 0.0, ms_best = 0.0;
  int tuned = 0;
};
std::mutex g_tune_mx;
std::map<std::tuple<int, int, int>, LaunchCfg> g_tune;

LaunchCfg tuned_cfg(int m, int a_dtype) {
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tune_mx);
  auto it = g_tune.find({dev, m, a_dtype});
  return it == g_tune.end() ? LaunchCfg{} : it->second;
}

hipError_t launch_upscale_cfg(const UpArgs& args, int a_dtype, hipStream_t st, const LaunchCfg& c) {
  if (args.m <= 8) return launch_upscale_small(args, a_dtype, st, c.lane_block);
  if (tiled_supports(args.m)) return launch_upscale_tiled(args, a_dtype, st, c.tiled_waves);
  return launch_upscale_ref(args, a_dtype, st);
}

// Plain FP64 upscaling of one homogeneous batch with the kernel suited to its
// m, in the tuned launch shape.
hipError_t launch_upscale_any(const UpArgs& args, int a_dtype, hipStream_t st) {
  return launch_upscale_cfg(args, a_dtype, st, tuned_cfg(args.m, a_dtype));
}
}  // namespace stomsfem

// Library-owned model (reduced basis).  All arrays live on `device`.
struct stomsfem_model {
  int kind = 0;  // 1 = reduced basis
  int device = 0;
  int ncx = 0, ncy = 0, m = 0, rmax = 8, KD = 0, PP = 0;
  int32_t* rK = nullptr;
  double* lambda = nullptr;
  double* Z = nullptr;
  double* phibar = nullptr;
  float* G32 = nullptr;
  double* G64 = nullptr;
  // learned surrogate (kind 2)
  int32_t* lv = nullptr;      // [M][4]
  float* params = nullptr;    // [M][NP]
  float* m1 = nullptr;
  float* m2 = nullptr;
  double* mu = nullptr;       // [M][10]
  double* sd = nullptr;
  double* sd_raw = nullptr;
  float* X = nullptr;         // [M][ntrain][4]
  float* T = nullptr;         // [M][ntrain][10]
  int64_t ntrain = 0;
  int64_t adam_t = 0;
  double box = 1.0;
  stomsfem_bump_family fam{};
  int32_t lv_max = -1;        // largest local-variable index
  int64_t* list = nullptr;    // fallback list
  int64_t list_cap = 0;
  int32_t family = 0;         // surrogate coefficient family (MLP_FAMILY_*)
  int32_t* fmap = nullptr;    // channels medium: feature per fine element [nc*m][nc*m]
  double* rw = nullptr;       // channels medium: [M][4] boundary-ring fractions of the local features
  int32_t nfeat = 0;
  double decades = 0.0;
  unsigned long long* counter = nullptr;
  // random interpolation (kind 3)
  int nn = 0;
  double lo = -1.0, hi = 1.0;
  int64_t rows = 0;           // table rows (tensor nodes of all patches)
  int64_t* off = nullptr;     // [M + 1]
  int32_t* nlv = nullptr;     // [M]
  double* table = nullptr;    // [rows][10]
  int64_t chunk = 0;          // pairs per plain-solve chunk
  double* blk = nullptr;      // [chunk][m][m] coefficient blocks
  double* xin = nullptr;      // [chunk][nxi] node random vectors
  int64_t* pairs = nullptr;   // [chunk]
  double* Sc = nullptr;       // [chunk][10]
  int32_t* stc = nullptr;     // [chunk]
  // sparse-grid collocation dictionaries (kind 4): rows, off, nlv, lv, table
  // as above; keys of the local points, increasing within each patch
  int64_t* keys = nullptr;    // [rows]
  int32_t sc_level = 0;
  // sparse-grid interpolation (kind 5): rows, off, nlv, lv, table, list and
  // the chunk buffers as for kind 3, plus the combination entries
  double* cb_coef = nullptr;
  uint32_t* cb_boff = nullptr;
  int32_t* cb_rows = nullptr;  // per k: entry offsets of the table rows
  double* sg_nodes = nullptr;  // [nb]
  int32_t sg_nb = 0, sg_kmax = 0;
  int32_t sg_lofs[SGI_LEVEL_MAX + 3] = {};
  int32_t sg_rofs[6] = {};
  // KL interpolation (kind 6; kind 7 = of the oversampled Petrov-Galerkin
  // stiffness: nine class tables of 16 entries, os_o cells of oversampling)
  int32_t os_o = 0;
  // reduced basis on oversampled patches (kind 9): m is the patch side, os_o
  // the oversampling, os_m the element side; online tables GO / GO32
  // [M][KD][RBO_PO] and corner values Pc [M][4][RBO_NF]
  int32_t os_m = 0;
  double* GO = nullptr;
  float* GO32 = nullptr;
  double* Pc = nullptr;
  // ordering of the calls that use the model's scratch buffers (OrderedUse)
  std::mutex order_mu;
  hipEvent_t order_ev = nullptr;
};

namespace {
RbOsArgs rb_os_args(const stomsfem_model* md) {
  RbOsArgs t{};
  t.ncx = md->ncx;
  t.ncy = md->ncy;
  t.m = md->os_m;
  t.o = md->os_o;
  t.Mp = md->m;
  t.rmax = md->rmax;
  t.KD = md->KD;
  t.PP = md->PP;
  t.KDo = md->KD;
  t.rK = md->rK;
  t.Z = md->Z;
  t.phibar = md->phibar;
  t.G64 = md->G64;
  t.GO = md->GO;
  t.GO32 = md->GO32;
  t.Pc = md->Pc;
  return t;
}

void model_release(stomsfem_model* md) {
  if (!md) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(md->device);
  hipDeviceSynchronize();
  hipFree(md->rK);
  hipFree(md->lambda);
  hipFree(md->Z);
  hipFree(md->phibar);
  hipFree(md->G32);
  hipFree(md->G64);
  hipFree(md->GO);
  hipFree(md->GO32);
  hipFree(md->Pc);
  hipFree(md->lv);
  hipFree(md->params);
  hipFree(md->m1);
  hipFree(md->m2);
  hipFree(md->mu);
  hipFree(md->sd);
  hipFree(md->sd_raw);
  hipFree(md->X);
  hipFree(md->T);
  hipFree(md->list);
  hipFree(md->counter);
  hipFree(md->off);
  hipFree(md->nlv);
  hipFree(md->table);
  hipFree(md->blk);
  hipFree(md->xin);
  hipFree(md->pairs);
  hipFree(md->Sc);
  hipFree(md->stc);
  hipFree(md->keys);
  hipFree(md->cb_coef);
  hipFree(md->cb_boff);
  hipFree(md->cb_rows);
  hipFree(md->sg_nodes);
  hipFree(md->fmap);
  hipFree(md->rw);
  if (md->order_ev) hipEventDestroy(md->order_ev);
  hipSetDevice(cur);
  delete md;
}
}  // namespace

extern "C" {

int stomsfem_version(void) { return STOMSFEM_ABI_VERSION; }

const char* stomsfem_last_error(void) { return g_last_error.c_str(); }

int stomsfem_coef_bumps(int64_t nsamples, int32_t nfine, const double* xi, int32_t nxi, int32_t g, double rho,
                        double eps, double base, double amp, double beta, void* a, int32_t a_dtype, void* stream) {
  if (nsamples < 0 || nfine < 1 || g < 1 || nxi < g * g) return fail(STOMSFEM_EINVAL, "coef_bumps: bad sizes");
  if (!(rho > 0.0) || !(eps > 0.0)) return fail(STOMSFEM_EINVAL, "coef_bumps: rho and eps must be > 0");
  if (a_dtype != STOMSFEM_F64 && a_dtype != STOMSFEM_F32) return fail(STOMSFEM_EINVAL, "coef_bumps: bad a_dtype");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(xi) || !device_ptr(a)) return fail(STOMSFEM_EINVAL, "coef_bumps: xi and a must be device pointers");
  hipError_t e = launch_coef_bumps(nsamples, nfine, xi, nxi, g, rho, eps, base, amp, beta, a, a_dtype,
                                   (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "coef_bumps launch");
}

int stomsfem_feature_map(int32_t nfine, int32_t nfeat, const int32_t* kind, const double* x0, const double* y0,
                         const double* size, int32_t* map, void* stream) {
  if (nfine < 1 || nfeat < 0 || nfeat > 1024) return fail(STOMSFEM_EINVAL, "feature_map: need nfine >= 1, 0 <= nfeat <= 1024");
  if (!device_ptr(map)) return fail(STOMSFEM_EINVAL, "feature_map: map must be a device pointer");
  if (nfeat > 0 && (!device_ptr(kind) || !device_ptr(x0) || !device_ptr(y0) || !device_ptr(size)))
    return fail(STOMSFEM_EINVAL, "feature_map: geometry arrays must be device pointers");
  hipError_t e = launch_feature_map(nfine, nfeat, kind, x0, y0, size, map, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "feature_map launch");
}

int stomsfem_coef_features(int64_t nsamples, int32_t nfine, const int32_t* map, int32_t nfeat, const double* xi,
                           int32_t nxi, double decades, void* a, int32_t a_dtype, void* stream) {
  if (nsamples < 0 || nfine < 1 || nfeat < 0 || nfeat > 1024 || nxi < nfeat)
    return fail(STOMSFEM_EINVAL, "coef_features: bad sizes");
  if (a_dtype != STOMSFEM_F64 && a_dtype != STOMSFEM_F32) return fail(STOMSFEM_EINVAL, "coef_features: bad a_dtype");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(map) || !device_ptr(a) || (nfeat > 0 && !device_ptr(xi)))
    return fail(STOMSFEM_EINVAL, "coef_features: map, xi and a must be device pointers");
  hipError_t e = launch_coef_features(nsamples, nfine, map, nfeat, xi, nxi, decades, a, a_dtype, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "coef_features launch");
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// One batch in STOMSFEM_PREC_F32_REFINE64: the mixed-precision kernel, then
// the FP64 kernels on the pairs it hands back (read synchronously).
static int upscale_refined(const stomsfem_batch& b, hipStream_t st) {
  UpArgs up = to_args(b);
  const int m = b.m;
  const int64_t chunk = std::min<int64_t>(
      up.npairs, std::max<int64_t>(256, std::min<int64_t>(65536, (int64_t{1} << 25) / ((int64_t)m * m))));
  const size_t off_list = 256;
  const size_t off_blk = off_list + align256(sizeof(int64_t) * (size_t)up.npairs);
  const size_t off_Sc = off_blk + align256(sizeof(double) * (size_t)chunk * m * m);
  const size_t off_stc = off_Sc + align256(sizeof(double) * 10 * (size_t)chunk);
  const size_t total = off_stc + align256(sizeof(int32_t) * (size_t)chunk);
  void* ws = nullptr;
  WorkspaceLease lease;
  int rc = lease.acquire(total, st, &ws);
  if (rc != STOMSFEM_OK) return rc;
  char* base = (char*)ws;
  auto* counter = (unsigned long long*)base;
  auto* list = (int64_t*)(base + off_list);
  auto* blk = (double*)(base + off_blk);
  auto* Sc = (double*)(base + off_Sc);
  auto* stc = (int32_t*)(base + off_stc);
  MixedArgs ma{};
  ma.up = up;
  ma.tol = STOMSFEM_REFINE_TOL;
  ma.max_iter = STOMSFEM_REFINE_MAXIT;
  ma.list = list;
  ma.count = counter;
  hipError_t e = launch_zero_u64(counter, st);
  if (e == hipSuccess) e = launch_upscale_mixed(ma, b.a_dtype, st);
  unsigned long long n = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&n, counter, sizeof(n), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "upscale (FP32 + FP64 refinement)");
  if (n > (unsigned long long)up.npairs) return fail(STOMSFEM_EHIP, "upscale: refinement fallback count out of range");
  g_refine_pairs += (uint64_t)up.npairs;
  g_refine_recomputed += n;
  for (int64_t start = 0; start < (int64_t)n && e == hipSuccess; start += chunk) {
    const int64_t cnt = std::min<int64_t>(chunk, (int64_t)n - start);
    e = launch_gather_blocks(up, b.a_dtype, list + start, cnt, blk, st);
    if (e == hipSuccess) {
      UpArgs u{};
      u.nsamples = cnt;
      u.ncx = u.ncy = 1;
      u.m = m;
      u.npairs = cnt;
      u.a = blk;
      u.S = Sc;
      u.status = stc;
      e = launch_upscale_any(u, STOMSFEM_F64, st);
    }
    if (e == hipSuccess) e = launch_scatter_pairs(list + start, cnt, Sc, stc, b.S, b.status, 1, st);
  }
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "upscale: FP64 recompute launch");
}

int stomsfem_upscale(const stomsfem_batch* batches, int32_t nbatch, int32_t precision, int32_t bc, void* stream) {
  if (nbatch < 0 || (nbatch > 0 && !batches)) return fail(STOMSFEM_EINVAL, "upscale: bad batch list");
  if (precision != STOMSFEM_PREC_F64 && precision != STOMSFEM_PREC_F32_REFINE64 && precision != STOMSFEM_PREC_AUTO)
    return fail(STOMSFEM_EINVAL, "upscale: precision must be STOMSFEM_PREC_F64, _F32_REFINE64 or _AUTO");
  if (bc != STOMSFEM_BC_LINEAR && bc != STOMSFEM_BC_OSCILLATORY)
    return fail(STOMSFEM_EINVAL, "upscale: bc must be STOMSFEM_BC_LINEAR or STOMSFEM_BC_OSCILLATORY");
  if (bc == STOMSFEM_BC_OSCILLATORY && precision == STOMSFEM_PREC_F32_REFINE64)
    return fail(STOMSFEM_EINVAL, "upscale: oscillatory boundary data are served by the FP64 reference kernel only");
  for (int i = 0; i < nbatch; ++i) {
    int rc = check_batch(batches[i], i);
    if (rc != STOMSFEM_OK) return rc;
    const int prec_i =
        precision == STOMSFEM_PREC_AUTO ? tuned_cfg(batches[i].m, batches[i].a_dtype).precision : precision;
    if (prec_i == STOMSFEM_PREC_F32_REFINE64 && batches[i].nsamples > 0) {
      if (batches[i].m > 32) return fail(STOMSFEM_EINVAL, "upscale: FP32 + refinement needs m <= 32");
      int dev = 0, maxlds = 0;
      hipGetDevice(&dev);
      hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
      if (upscale_mixed_lds_bytes(batches[i].m) + 256 > (size_t)maxlds)
        return fail(STOMSFEM_EINVAL, "upscale: FP32 + refinement needs " +
                                         std::to_string(upscale_mixed_lds_bytes(batches[i].m)) +
                                         " bytes of LDS per workgroup; the device allows " + std::to_string(maxlds));
    }
  }
  for (int i = 0; i < nbatch; ++i) {
    const stomsfem_batch& b = batches[i];
    if (b.nsamples == 0) continue;
    if (bc == STOMSFEM_BC_OSCILLATORY) {
      UpArgs up = to_args(b);
      up.bc = STOMSFEM_BC_OSCILLATORY;
      hipError_t e = launch_upscale_ref(up, b.a_dtype, (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "upscale launch");
      continue;
    }
    const int prec_b = precision == STOMSFEM_PREC_AUTO ? tuned_cfg(b.m, b.a_dtype).precision : precision;
    if (prec_b == STOMSFEM_PREC_F32_REFINE64) {
      int rc = upscale_refined(b, (hipStream_t)stream);
      if (rc != STOMSFEM_OK) return rc;
      continue;
    }
    hipError_t e = launch_upscale_any(to_args(b), b.a_dtype, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "upscale launch");
  }
  return STOMSFEM_OK;
}

int stomsfem_upscale_reference(const stomsfem_batch* batch, int32_t bc, void* stream) {
  if (!batch) return fail(STOMSFEM_EINVAL, "upscale_reference: NULL batch");
  if (bc != STOMSFEM_BC_LINEAR && bc != STOMSFEM_BC_OSCILLATORY)
    return fail(STOMSFEM_EINVAL, "upscale_reference: bc must be STOMSFEM_BC_LINEAR or STOMSFEM_BC_OSCILLATORY");
  int rc = check_batch(*batch, 0);
  if (rc != STOMSFEM_OK) return rc;
  if (batch->nsamples == 0) return STOMSFEM_OK;
  UpArgs up = to_args(*batch);
  up.bc = bc;
  hipError_t e = launch_upscale_ref(up, batch->a_dtype, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "upscale_reference launch");
}

int stomsfem_element_loads(int32_t ncx, int32_t ncy, const double* f, double* load, void* stream) {
  if (ncx < 1 || ncy < 1 || (int64_t)ncx * ncy > (1 << 24))
    return fail(STOMSFEM_EINVAL, "element_loads: ncx, ncy must be >= 1 (at most 2^24 elements)");
  if (!f) return fail(STOMSFEM_EINVAL, "element_loads: f is NULL");
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(f[i])) return fail(STOMSFEM_EINVAL, "element_loads: f must be finite");
  if (!device_ptr(load)) return fail(STOMSFEM_EINVAL, "element_loads: load is not a device pointer");
  hipError_t e = launch_element_loads(ncx, ncy, f, load, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "element_loads launch");
}

int stomsfem_upscale_queue(const stomsfem_batch* batches, int32_t nbatch, void* stream) {
  if (nbatch < 1 || !batches) return fail(STOMSFEM_EINVAL, "upscale_queue: need at least one batch");
  if (nbatch > queue_max_batches())
    return fail(STOMSFEM_EINVAL, "upscale_queue: at most " + std::to_string(queue_max_batches()) + " batches");
  std::vector<UpArgs> up;
  int64_t pairs = 0;
  for (int i = 0; i < nbatch; ++i) {
    int rc = check_batch(batches[i], i);
    if (rc != STOMSFEM_OK) return rc;
    if (!queue_supports(batches[i].m))
      return fail(STOMSFEM_EINVAL, "upscale_queue: batch " + std::to_string(i) + ": m must be 8, 16 or 32");
    if (batches[i].a_dtype != batches[0].a_dtype)
      return fail(STOMSFEM_EINVAL, "upscale_queue: every batch must have the same a_dtype");
    up.push_back(to_args(batches[i]));
    pairs += up.back().npairs;
  }
  if (pairs == 0) return STOMSFEM_OK;
  WorkspaceLease lease;
  void* ws = nullptr;
  int rc = lease.acquire(256, (hipStream_t)stream, &ws);
  if (rc != STOMSFEM_OK) return rc;
  hipError_t e = launch_upscale_queue(up.data(), nbatch, batches[0].a_dtype, (unsigned long long*)ws,
                                      (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "upscale_queue launch");
}

int stomsfem_coarse_solve(int32_t ncx, int32_t ncy, int64_t nsamples, const double* S, const double* load,
                          double* U, double* qoi_mean, double* qoi_var, int32_t* status, void* stream) {
  if (ncx < 1 || ncy < 1 || nsamples < 0) return fail(STOMSFEM_EINVAL, "coarse_solve: bad sizes");
  if (ncx > 1024 || ncy > 1024) return fail(STOMSFEM_EINVAL, "coarse_solve: ncx, ncy must be <= 1024");
  if (coarse_lds_bytes(ncx, false) > 64 * 1024) return fail(STOMSFEM_EINVAL, "coarse_solve: ncx too large for the LDS window");
  const int nU = (ncx - 1) * (ncy - 1);
  if (nU == 0) return STOMSFEM_OK;
  if (nsamples > 0 && (!device_ptr(S) || !device_ptr(U)))
    return fail(STOMSFEM_EINVAL, "coarse_solve: S and U must be device pointers");
  if (load && !device_ptr(load)) return fail(STOMSFEM_EINVAL, "coarse_solve: load must be a device pointer");
  if ((qoi_mean && !device_ptr(qoi_mean)) || (qoi_var && !device_ptr(qoi_var)))
    return fail(STOMSFEM_EINVAL, "coarse_solve: qoi outputs must be device pointers");
  if (status && !device_ptr(status)) return fail(STOMSFEM_EINVAL, "coarse_solve: status must be a device pointer");
  void* work = nullptr;
  WorkspaceLease lease;
  if (nsamples > 0) {
    int rc = lease.acquire(sizeof(double) * (size_t)coarse_work_doubles(ncx, ncy, nsamples), (hipStream_t)stream,
                           &work);
    if (rc != STOMSFEM_OK) return rc;
  }
  hipError_t e = launch_coarse(ncx, ncy, nsamples, S, load, U, qoi_mean, qoi_var, status, (double*)work,
                               (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "coarse_solve launch");
}

// ---------------------------------------------------------------------------
// Coarse solve without allocation.  Its factor workspace is a fixed array in
// device memory that every GPU running the library holds from module load to
// process end.  `scratch` is a host-side stand-in: its device address on the
// current device comes from hipGetSymbolAddress (once per device, kept in
// g_scratch_ptr) and only that address is ever handed to kernels.
// ---------------------------------------------------------------------------
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = int64_t{8} << 20;  // 64 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};  // device -> address of `scratch` there (no host allocation)

int scratch_device_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(STOMSFEM_EINVAL, "coarse_solve_noalloc: device index too large");
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(STOMSFEM_EHIP, std::string("coarse_solve_noalloc: hipGetSymbolAddress of the scratch array failed: ") +
                                     hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return STOMSFEM_OK;
}
}  // namespace

int stomsfem_coarse_solve_noalloc(int32_t ncx, int32_t ncy, int64_t nsamples, const double* S, const double* load,
                                  double* U, double* qoi_mean, double* qoi_var, int32_t* status, void* stream) {
  if (ncx < 1 || ncy < 1 || nsamples < 0) return fail(STOMSFEM_EINVAL, "coarse_solve_noalloc: bad sizes");
  if (ncx > 1024 || ncy > 1024) return fail(STOMSFEM_EINVAL, "coarse_solve_noalloc: ncx, ncy must be <= 1024");
  if (coarse_lds_bytes(ncx, false) > 64 * 1024)
    return fail(STOMSFEM_EINVAL, "coarse_solve_noalloc: ncx too large for the LDS window");
  const int64_t nU = (int64_t)(ncx - 1) * (ncy - 1);
  if (nU == 0) return STOMSFEM_OK;
  const int64_t per = nU * (ncx + 1) + 1;
  if (per > NOALLOC_SCRATCH_DOUBLES || 2 * nU > NOALLOC_SCRATCH_DOUBLES)
    return fail(STOMSFEM_EINVAL, "coarse_solve_noalloc: one sample of a " + std::to_string(ncx) + " x " +
                                     std::to_string(ncy) + " coarse mesh needs " + std::to_string(8 * per) +
                                     " bytes of scratch, more than the " +
                                     std::to_string(8 * NOALLOC_SCRATCH_DOUBLES) + " bytes the library holds");
  if (nsamples > 0 && (!device_ptr(S) || !device_ptr(U)))
    return fail(STOMSFEM_EINVAL, "coarse_solve_noalloc: S and U must be device pointers");
  if (load && !device_ptr(load)) return fail(STOMSFEM_EINVAL, "coarse_solve_noalloc: load must be a device pointer");
  if ((qoi_mean && !device_ptr(qoi_mean)) || (qoi_var && !device_ptr(qoi_var)))
    return fail(STOMSFEM_EINVAL, "coarse_solve_noalloc: qoi outputs must be device pointers");
  if (status && !device_ptr(status))
    return fail(STOMSFEM_EINVAL, "coarse_solve_noalloc: status must be a device pointer");
  double* work = nullptr;
  int rc = scratch_device_ptr(&work);
  if (rc != STOMSFEM_OK) return rc;
  hipError_t e = launch_coarse_capped(ncx, ncy, nsamples, S, load, U, qoi_mean, qoi_var, status, work,
                                      NOALLOC_SCRATCH_DOUBLES, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "coarse_solve_noalloc launch");
}

int stomsfem_fine_solve_pcg(const double* a, int32_t nfine, int64_t nsamples, double tol, int32_t max_iter,
                            double* u, int32_t* iters, int32_t* status, void* stream) {
  if (nfine < 2 || nfine > 8192 || nsamples < 0) return fail(STOMSFEM_EINVAL, "fine_solve_pcg: need 2 <= nfine <= 8192");
  if (!(tol > 0.0) || max_iter < 1) return fail(STOMSFEM_EINVAL, "fine_solve_pcg: need tol > 0 and max_iter >= 1");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(a) || !device_ptr(u)) return fail(STOMSFEM_EINVAL, "fine_solve_pcg: a and u must be device pointers");
  if ((status && !device_ptr(status)) || (iters && !device_ptr(iters)))
    return fail(STOMSFEM_EINVAL, "fine_solve_pcg: status and iters must be device pointers");
  const int64_t per = fine_pcg_doubles_per_sample(nfine);
  // samples per chunk: about 4 GiB of vectors, at most 64
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>({nsamples, (int64_t)64, (int64_t{1} << 29) / per}));
  hipStream_t st = (hipStream_t)stream;
  void* ws = nullptr;
  WorkspaceLease lease;
  int rc = lease.acquire(sizeof(double) * (size_t)per * chunk + sizeof(int32_t) * (size_t)chunk, st, &ws);
  if (rc != STOMSFEM_OK) return rc;
  double* work = (double*)ws;
  int32_t* it_scratch = (int32_t*)(work + per * chunk);
  const int64_t ncell = (int64_t)nfine * nfine, nU = (int64_t)(nfine - 1) * (nfine - 1);
  for (int64_t start = 0; start < nsamples; start += chunk) {
    const int64_t cnt = std::min(chunk, nsamples - start);
    hipError_t e = launch_fine_pcg(a + start * ncell, nfine, cnt, tol, max_iter, u + start * nU,
                                   iters ? iters + start : it_scratch, status ? status + start : nullptr, work, st);
    if (e != hipSuccess) return hip_fail(e, "fine_solve_pcg");
  }
  return STOMSFEM_OK;
}

int stomsfem_fine_solve(const double* a, int32_t nfine, int64_t nsamples, double* u, int32_t* status,
                        void* stream) {
  if (nfine > 64 && nfine <= 8192 && nsamples >= 0)  // beyond the direct solver's band window
    return stomsfem_fine_solve_pcg(a, nfine, nsamples, STOMSFEM_FINE_PCG_TOL, STOMSFEM_FINE_PCG_MAXIT, u, nullptr,
                                   status, stream);
  if (nfine < 2 || nfine > 64 || nsamples < 0) return fail(STOMSFEM_EINVAL, "fine_solve: need 2 <= nfine <= 8192");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(a) || !device_ptr(u)) return fail(STOMSFEM_EINVAL, "fine_solve: a and u must be device pointers");
  if (status && !device_ptr(status)) return fail(STOMSFEM_EINVAL, "fine_solve: status must be a device pointer");
  // the fine FEM is the coarse system of the m = 1 upscaled elements
  // a_e K_Q1 on the nfine x nfine mesh, with the load h^2/4 per element node
  const int64_t per = (int64_t)nfine * nfine, nU = (int64_t)(nfine - 1) * (nfine - 1);
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nsamples, (int64_t{1} << 27) / (per * 80)));
  const size_t s_doubles = (size_t)chunk * per * 10;
  const size_t w_doubles = (size_t)coarse_work_doubles(nfine, nfine, chunk);
  void* ws = nullptr;
  hipStream_t st = (hipStream_t)stream;
  WorkspaceLease lease;
  int rc = lease.acquire(sizeof(double) * (s_doubles + w_doubles), st, &ws);
  if (rc != STOMSFEM_OK) return rc;
  double* Sbuf = (double*)ws;
  double* work = Sbuf + s_doubles;
  for (int64_t start = 0; start < nsamples; start += chunk) {
    const int64_t cnt = std::min(chunk, nsamples - start);
    UpArgs up{};
    up.nsamples = cnt;
    up.ncx = up.ncy = nfine;
    up.m = 1;
    up.npairs = cnt * per;
    up.a = a + start * per;
    up.S = Sbuf;
    up.status = nullptr;
    hipError_t e = launch_upscale_any(up, STOMSFEM_F64, st);
    if (e == hipSuccess)
      e = launch_coarse(nfine, nfine, cnt, Sbuf, nullptr, u + start * nU, nullptr, nullptr,
                        status ? status + start : nullptr, work, st);
    if (e != hipSuccess) return hip_fail(e, "fine_solve launch");
  }
  return STOMSFEM_OK;
}

int stomsfem_two_level_mc(const double* U_H, int64_t n_H, const double* U_Hh, const double* u_fine, int64_t n_h,
                          int32_t nc, int32_t m, double* mean, double* var_H, double* var_d, void* stream) {
  if (n_H < 1 || n_h < 1 || nc < 2 || m < 1 || (int64_t)nc * m > 65536)
    return fail(STOMSFEM_EINVAL, "two_level_mc: need n_H, n_h >= 1, nc >= 2, m >= 1");
  if (!device_ptr(U_H) || !device_ptr(U_Hh) || !device_ptr(u_fine))
    return fail(STOMSFEM_EINVAL, "two_level_mc: U_H, U_Hh and u_fine must be device pointers");
  if ((mean && !device_ptr(mean)) || (var_H && !device_ptr(var_H)) || (var_d && !device_ptr(var_d)))
    return fail(STOMSFEM_EINVAL, "two_level_mc: outputs must be device pointers");
  hipError_t e = launch_two_level(U_H, n_H, U_Hh, u_fine, n_h, nc, m, mean, var_H, var_d, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "two_level_mc launch");
}

int stomsfem_coef_gauss(int64_t nsamples, int32_t nfine, int32_t nterms, const double* z, const double* u, double l1,
                        double l2, double* beta, double* kappa, void* stream) {
  if (nsamples < 0 || nfine < 1 || nterms < 1 || nterms > 1024 || !(l1 > 0) || !(l2 > 0))
    return fail(STOMSFEM_EINVAL, "coef_gauss: need nfine >= 1, 1 <= nterms <= 1024, l1, l2 > 0");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(z) || !device_ptr(u) || !device_ptr(kappa) || (beta && !device_ptr(beta)))
    return fail(STOMSFEM_EINVAL, "coef_gauss: z, u, kappa (and beta) must be device pointers");
  hipError_t e = launch_gauss_field(nsamples, nfine, nterms, z, u, l1, l2, beta, kappa, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "coef_gauss launch");
}

int stomsfem_local_kl(int32_t m, double h, double l1, double l2, int32_t K, double* mu, double* modes,
                      double* captured) {
  if (m < 1 || m > 64 || K < 1 || K > 16 || K > m * m || !(h > 0) || !(l1 > 0) || !(l2 > 0))
    return fail(STOMSFEM_EINVAL, "local_kl: need 1 <= m <= 64, 1 <= K <= min(16, m*m), h, l1, l2 > 0");
  if (!mu || !modes) return fail(STOMSFEM_EINVAL, "local_kl: NULL output");
  local_kl_modes(m, h, l1, l2, K, mu, modes, captured);
  return STOMSFEM_OK;
}

static int kl_project_any(const char* name, int64_t nsamples, int32_t nc, int32_t m, int32_t o, const double* beta,
                          int32_t K, const double* mu, const double* modes, double box, double* xi, int32_t* outside,
                          uint64_t* count, void* stream) {
  const int64_t P = (int64_t)m + 2 * (int64_t)o;
  if (nsamples < 0 || nc < 1 || m < 1 || o < 0 || P > (int64_t)nc * m || K < 1 || K > 16 || K > P * P || !(box > 0))
    return fail(STOMSFEM_EINVAL, std::string(name) +
                                     ": need nc, m >= 1, 0 <= oversample, m + 2 oversample <= nc m, "
                                     "1 <= K <= min(16, (m + 2 oversample)^2), box > 0");
  if (!device_ptr(beta) || !device_ptr(mu) || !device_ptr(modes) || !device_ptr(xi) ||
      (outside && !device_ptr(outside)) || (count && !device_ptr(count)))
    return fail(STOMSFEM_EINVAL, std::string(name) + ": arrays must be device pointers");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (count) e = launch_zero_u64((unsigned long long*)count, st);
  if (e == hipSuccess)
    e = launch_kl_project(nsamples * (int64_t)nc * nc, nc, m, o, K, beta, mu, modes, box, xi, outside,
                          (unsigned long long*)count, st);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, (std::string(name) + " launch").c_str());
}

int stomsfem_kl_project(int64_t nsamples, int32_t nc, int32_t m, const double* beta, int32_t K, const double* mu,
                        const double* modes, double box, double* xi, int32_t* outside, uint64_t* count,
                        void* stream) {
  return kl_project_any("kl_project", nsamples, nc, m, 0, beta, K, mu, modes, box, xi, outside, count, stream);
}

int stomsfem_kl_project_patches(int64_t nsamples, int32_t nc, int32_t m, int32_t oversample, const double* beta,
                                int32_t K, const double* mu, const double* modes, double box, double* xi,
                                int32_t* outside, uint64_t* count, void* stream) {
  return kl_project_any("kl_project_patches", nsamples, nc, m, oversample, beta, K, mu, modes, box, xi, outside,
                        count, stream);
}

int stomsfem_kl_blocks(int64_t npairs, int32_t m, int32_t Kuse, int32_t K, const double* xi, const double* mu,
                       const double* modes, double* blocks, void* stream) {
  if (npairs < 0 || m < 1 || K < 1 || K > 16 || Kuse < 0 || Kuse > K)
    return fail(STOMSFEM_EINVAL, "kl_blocks: need m >= 1, 1 <= K <= 16, 0 <= Kuse <= K");
  if (npairs == 0) return STOMSFEM_OK;
  if (!device_ptr(xi) || !device_ptr(mu) || !device_ptr(modes) || !device_ptr(blocks))
    return fail(STOMSFEM_EINVAL, "kl_blocks: arrays must be device pointers");
  hipError_t e = launch_kl_blocks(npairs, m, Kuse, K, xi, mu, modes, blocks, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "kl_blocks launch");
}

int stomsfem_kl_interp_build(int32_t ncx, int32_t ncy, int32_t m, int32_t K, const double* mu, const double* modes,
                             int32_t nnodes, double box, stomsfem_model** model, void* stream) {
  if (!model) return fail(STOMSFEM_EINVAL, "kl_interp_build: NULL model");
  *model = nullptr;
  if (ncx < 1 || ncy < 1 || m < 1 || m > 48 || K < 1 || K > RI_KMAX || nnodes < RI_NN_MIN || nnodes > RI_NN_MAX ||
      !(box > 0))
    return fail(STOMSFEM_EINVAL, "kl_interp_build: need 1 <= m <= 48, 1 <= K <= 4, 2 <= nnodes <= 9, box > 0");
  if (!device_ptr(mu) || !device_ptr(modes)) return fail(STOMSFEM_EINVAL, "kl_interp_build: mu and modes on device");
  const int Mc = ncx * ncy;
  int64_t rows = 1;
  for (int i = 0; i < K; ++i) rows *= nnodes;
  hipStream_t st = (hipStream_t)stream;
  auto* md = new stomsfem_model();
  md->kind = 6;
  hipGetDevice(&md->device);
  md->ncx = ncx;
  md->ncy = ncy;
  md->m = m;
  md->nn = nnodes;
  md->lo = -box;
  md->hi = box;
  md->rows = rows;
  md->chunk = std::max<int64_t>(256, std::min<int64_t>(65536, (int64_t{1} << 25) / ((int64_t)m * m)));
  hipError_t e = hipSuccess;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  };
  double* xin = nullptr;
  double* blk = nullptr;
  A((void**)&md->lv, sizeof(int32_t) * Mc * RI_KMAX);
  A((void**)&md->nlv, sizeof(int32_t) * Mc);
  A((void**)&md->off, sizeof(int64_t) * (Mc + 1));
  A((void**)&md->table, sizeof(double) * (size_t)rows * 10);
  A((void**)&md->counter, sizeof(unsigned long long));
  A((void**)&md->blk, sizeof(double) * (size_t)md->chunk * m * m);
  A((void**)&md->Sc, sizeof(double) * (size_t)md->chunk * 10);
  A((void**)&md->stc, sizeof(int32_t) * (size_t)md->chunk);
  A((void**)&xin, sizeof(double) * (size_t)rows * K);
  A((void**)&blk, sizeof(double) * (size_t)rows * m * m);
  int32_t* stn = nullptr;
  A((void**)&stn, sizeof(int32_t) * (size_t)rows);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    hipFree(xin);
    hipFree(blk);
    hipFree(stn);
    model_release(md);
    return fail(STOMSFEM_ENOMEM, "kl_interp_build: device allocation failed");
  }
  // every element reads the one table: local variables = its own K parameters
  std::vector<int32_t> lv((size_t)Mc * RI_KMAX, -1), nlv(Mc, K);
  std::vector<int64_t> off(Mc + 1, 0);
  for (int p = 0; p < Mc; ++p)
    for (int k = 0; k < K; ++k) lv[(size_t)p * RI_KMAX + k] = p * K + k;
  off[Mc] = rows;
  std::vector<double> xh((size_t)rows * K);
  for (int64_t r = 0; r < rows; ++r) {
    int64_t c = r;
    for (int v = K - 1; v >= 0; --v) {  // variable 0 slowest
      const int d = (int)(c % nnodes);
      c /= nnodes;
      xh[(size_t)r * K + v] = -box + (std::cos(M_PI * (double)d / (double)(nnodes - 1)) + 1.0) * box;
    }
  }
  e = hipMemcpy(md->lv, lv.data(), sizeof(int32_t) * lv.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->nlv, nlv.data(), sizeof(int32_t) * Mc, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->off, off.data(), sizeof(int64_t) * (Mc + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(xin, xh.data(), sizeof(double) * xh.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_kl_blocks(rows, m, K, K, xin, mu, modes, blk, st);
  if (e == hipSuccess) {
    UpArgs u{};
    u.nsamples = rows;
    u.ncx = u.ncy = 1;
    u.m = m;
    u.npairs = rows;
    u.a = blk;
    u.S = md->table;
    u.status = stn;
    e = launch_upscale_any(u, STOMSFEM_F64, st);
  }
  std::vector<int32_t> sth((size_t)rows);
  if (e == hipSuccess) e = hipMemcpyAsync(sth.data(), stn, sizeof(int32_t) * rows, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(xin);
  hipFree(blk);
  hipFree(stn);
  if (e != hipSuccess) {
    model_release(md);
    return hip_fail(e, "kl_interp_build");
  }
  for (int64_t r = 0; r < rows; ++r)
    if (sth[(size_t)r] != 0) {
      model_release(md);
      return fail(STOMSFEM_ENOTSPD, "kl_interp_build: a cell problem at a node is not positive definite");
    }
  md->lv_max = K;  // parameters per element
  *model = md;
  return STOMSFEM_OK;
}

// The level-L sparse grid in k = 1..4 variables (k = 0: the one empty
// point), the one-dimensional nodes of every level (level i at lofs[i]) and
// Smolyak's combination entries (coefficient, basis offsets) per k, grouped
// by the table row of their node, with per-k row offsets; `missing` is set if
// a tensor node of the combination is not a grid node.  Entries padded by
// SGI_BATCH - 1 for the kernel's batched reads.
struct SgiComb {
  std::vector<int32_t> gdig[RI_KMAX + 1];
  int64_t npts[RI_KMAX + 1] = {1, 0, 0, 0, 0};
  int32_t lofs[SGI_LEVEL_MAX + 3] = {};
  std::vector<double> nodes;
  std::vector<double> cc;
  std::vector<uint32_t> cbo;
  std::vector<int32_t> rows_all;
  int32_t rofs[6] = {};
  bool missing = false;
  int D = 1;
};

static void sgi_combination(int level, SgiComb& C) {
  const int D = sc_digit_base(level);
  C.D = D;
  auto& gdig = C.gdig;
  auto& npts = C.npts;
  auto& lofs = C.lofs;
  auto& nodes = C.nodes;
  auto& cc = C.cc;
  auto& cbo = C.cbo;
  auto& rows_all = C.rows_all;
  auto& rofs = C.rofs;
  bool missing = false;
  // the level-L grid in k variables (k = 1..4; k = 0: the one empty point)
  for (int k = 1; k <= RI_KMAX; ++k) {
    std::vector<double> gw;
    sc_build_grid(k, level, gdig[k], gw);
    npts[k] = (int64_t)gw.size();
  }
  // one-dimensional nodes of every level, level i at lofs[i]
  nodes.assign(1, 0.0);
  for (int i = 2; i <= level + 1; ++i) {
    const int n = (1 << (i - 1)) + 1;
    lofs[i] = (int32_t)nodes.size();
    for (int j = 0; j < n; ++j) nodes.push_back(std::cos(M_PI * (double)j / (double)(n - 1)));
  }
  // combination entries per k: (coefficient, basis offsets), grouped by the
  // table row of their node; per k the row offsets into the entries
  for (int k = 0; k <= RI_KMAX; ++k) {
    rofs[k] = (int32_t)rows_all.size();
    if (k == 0) {
      rows_all.push_back((int32_t)cc.size());
      cc.push_back(1.0);
      cbo.push_back(0u);
      rows_all.push_back((int32_t)cc.size());
      continue;
    }
    std::vector<std::vector<std::pair<double, uint32_t>>> byrow((size_t)npts[k]);
    std::map<std::vector<int32_t>, int32_t> rowof;
    for (int64_t r = 0; r < npts[k]; ++r)
      rowof[std::vector<int32_t>(gdig[k].begin() + r * k, gdig[k].begin() + (r + 1) * k)] = (int32_t)r;
    std::vector<int32_t> dg(k);
    std::vector<int> pos(k);
    sc_smolyak_terms(k, level, [&](double c, const std::vector<int>& idx) {
      for (int d = 0; d < k; ++d) pos[d] = 0;
      while (true) {
        uint32_t bo = 0;
        for (int d = 0; d < k; ++d) {
          const int n = idx[d] == 1 ? 1 : (1 << (idx[d] - 1)) + 1;
          dg[d] = n == 1 ? D / 2 : pos[d] * (D / (n - 1));
          bo |= (uint32_t)(lofs[idx[d]] + pos[d]) << (8 * d);
        }
        const auto it = rowof.find(dg);
        missing = missing || it == rowof.end();
        byrow[it == rowof.end() ? 0 : it->second].emplace_back(c, bo);
        int d = k - 1;
        while (d >= 0 && ++pos[d] == (idx[d] == 1 ? 1 : (1 << (idx[d] - 1)) + 1)) pos[d--] = 0;
        if (d < 0) break;
      }
    });
    for (int64_t r = 0; r < npts[k]; ++r) {
      rows_all.push_back((int32_t)cc.size());
      for (const auto& en : byrow[(size_t)r]) {
        cc.push_back(en.first);
        cbo.push_back(en.second);
      }
    }
    rows_all.push_back((int32_t)cc.size());
  }
  rofs[RI_KMAX + 1] = (int32_t)rows_all.size();
  C.missing = missing;
  cc.insert(cc.end(), SGI_BATCH - 1, 0.0);
  cbo.insert(cbo.end(), SGI_BATCH - 1, 0u);
}

// The nine class tables of an oversampled KL interpolation model (kinds 7,
// 8): md->table [9][rows][16] from the node parameters xin (device [rows][K]):
// the truncated local KL on the patch (nblk: device [rows][P][P] scratch),
// placed in 3 x 3-element meshes at each class, the oversampling kernels, the
// class element's entries; statuses into stn (device [9 rows]).
static hipError_t os_class_tables(stomsfem_model* md, int64_t rows, int K, const double* xin, const double* mu,
                                  const double* modes, double* nblk, int32_t* stn, hipStream_t st) {
  const int m = md->m, o = md->os_o, P = m + 2 * o;
  hipError_t e = launch_kl_blocks(rows, P, K, K, xin, mu, modes, nblk, st);
  for (int c = 0; c < 9 && e == hipSuccess; ++c) {
    const int cx = c % 3, cy = c / 3;
    for (int64_t start = 0; start < rows && e == hipSuccess; start += md->chunk) {
      const int64_t cnt = std::min<int64_t>(md->chunk, rows - start);
      e = launch_embed_patch(cnt, m, o, cx, cy, nblk + start * P * P, md->blk, st);
      if (e == hipSuccess) {
        UpArgs u{};
        u.nsamples = cnt;
        u.ncx = u.ncy = 3;
        u.m = m;
        u.npairs = cnt * 9;
        u.a = md->blk;
        u.S = md->Sc;
        u.status = md->stc;
        e = launch_upscale_os(u, o, STOMSFEM_F64, st);
      }
      if (e == hipSuccess)
        e = launch_pick_class(cnt, cx, cy, md->Sc, md->stc, md->table + (c * rows + start) * 16,
                              stn + c * rows + start, st);
    }
  }
  return e;
}

// Common part of the oversampled KL interpolation builds (kinds 7 and 8):
// md carries the mesh, m, os_o, lo/hi and rows (nodes per class); xh holds
// the node parameters [rows][K].  Allocates the model buffers, sets every
// element's table offset from its class, computes the nine class tables and
// checks the node solves.  Releases md and reports on failure.
static int os_kl_model_finish(stomsfem_model* md, int K, const std::vector<double>& xh, const double* mu,
                              const double* modes, hipStream_t st, const char* name) {
  const int ncx = md->ncx, ncy = md->ncy, m = md->m, o = md->os_o, P = m + 2 * o, Mc = ncx * ncy;
  const int64_t rows = md->rows;
  md->chunk = std::max<int64_t>(64, std::min<int64_t>(16384, (int64_t{1} << 22) / (9 * (int64_t)m * m)));
  hipError_t e = hipSuccess;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  };
  double* xin = nullptr;
  double* nblk = nullptr;
  int32_t* stn = nullptr;
  A((void**)&md->lv, sizeof(int32_t) * Mc * RI_KMAX);
  A((void**)&md->nlv, sizeof(int32_t) * Mc);
  A((void**)&md->off, sizeof(int64_t) * (Mc + 1));
  A((void**)&md->table, sizeof(double) * (size_t)rows * 9 * 16);
  A((void**)&md->counter, sizeof(unsigned long long));
  A((void**)&md->blk, sizeof(double) * (size_t)md->chunk * 9 * m * m);
  A((void**)&md->Sc, sizeof(double) * (size_t)md->chunk * 9 * 16);
  A((void**)&md->stc, sizeof(int32_t) * (size_t)md->chunk * 9);
  A((void**)&xin, sizeof(double) * (size_t)rows * K);
  A((void**)&nblk, sizeof(double) * (size_t)rows * P * P);
  A((void**)&stn, sizeof(int32_t) * (size_t)rows * 9);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    hipFree(xin);
    hipFree(nblk);
    hipFree(stn);
    model_release(md);
    return fail(STOMSFEM_ENOMEM, std::string(name) + ": device allocation failed");
  }
  // every element reads the table of its class with its own K parameters
  auto cls = [&](int k, int nc) {
    const int nf = nc * m;
    int x0 = k * m - o;
    if (x0 > nf - P) x0 = nf - P;
    if (x0 < 0) x0 = 0;
    return (k * m - x0) / o;
  };
  std::vector<int32_t> lv((size_t)Mc * RI_KMAX, -1), nlv(Mc, K);
  std::vector<int64_t> off(Mc + 1, 0);
  for (int p = 0; p < Mc; ++p) {
    for (int k = 0; k < K; ++k) lv[(size_t)p * RI_KMAX + k] = p * K + k;
    off[p] = (int64_t)(cls(p / ncx, ncy) * 3 + cls(p % ncx, ncx)) * rows;
  }
  off[Mc] = 9 * rows;
  e = hipMemcpy(md->lv, lv.data(), sizeof(int32_t) * lv.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->nlv, nlv.data(), sizeof(int32_t) * Mc, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->off, off.data(), sizeof(int64_t) * (Mc + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(xin, xh.data(), sizeof(double) * xh.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = os_class_tables(md, rows, K, xin, mu, modes, nblk, stn, st);
  std::vector<int32_t> sth((size_t)rows * 9);
  if (e == hipSuccess) e = hipMemcpyAsync(sth.data(), stn, sizeof(int32_t) * rows * 9, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(xin);
  hipFree(nblk);
  hipFree(stn);
  if (e != hipSuccess) {
    model_release(md);
    return hip_fail(e, name);
  }
  for (int64_t r = 0; r < rows * 9; ++r)
    if (sth[(size_t)r] != 0) {
      model_release(md);
      return fail(STOMSFEM_ENOTSPD, std::string(name) + ": a cell problem at a node failed");
    }
  md->lv_max = K;
  return STOMSFEM_OK;
}

static stomsfem_model* os_kl_model(int kind, int ncx, int ncy, int m, int o, double box, int64_t rows) {
  auto* md = new stomsfem_model();
  md->kind = kind;
  hipGetDevice(&md->device);
  md->ncx = ncx;
  md->ncy = ncy;
  md->m = m;
  md->os_o = o;
  md->lo = -box;
  md->hi = box;
  md->rows = rows;
  return md;
}

int stomsfem_kl_interp_os_build(int32_t ncx, int32_t ncy, int32_t m, int32_t oversample, int32_t K,
                                const double* mu, const double* modes, int32_t nnodes, double box,
                                stomsfem_model** model, void* stream) {
  if (!model) return fail(STOMSFEM_EINVAL, "kl_interp_os_build: NULL model");
  *model = nullptr;
  const int o = oversample, P = m + 2 * oversample;
  if (ncx < 1 || ncx != ncy || m < 1 || o < 1 || o > m || !upscale_os_supports(m, o) || P > ncx * m ||
      K < 1 || K > RI_KMAX || nnodes < RI_NN_MIN || nnodes > RI_NN_MAX || !(box > 0))
    return fail(STOMSFEM_EINVAL,
                "kl_interp_os_build: need a square mesh, 1 <= oversample <= m, m + 2 oversample <= 64 and <= the "
                "domain, "
                "1 <= K <= 4, 2 <= nnodes <= 9, box > 0");
  if (!device_ptr(mu) || !device_ptr(modes))
    return fail(STOMSFEM_EINVAL, "kl_interp_os_build: mu and modes on device");
  int64_t rows = 1;
  for (int i = 0; i < K; ++i) rows *= nnodes;
  auto* md = os_kl_model(7, ncx, ncy, m, o, box, rows);
  md->nn = nnodes;
  // tensor Lobatto nodes, variable 0 slowest
  std::vector<double> xh((size_t)rows * K);
  for (int64_t r = 0; r < rows; ++r) {
    int64_t c = r;
    for (int v = K - 1; v >= 0; --v) {
      const int d = (int)(c % nnodes);
      c /= nnodes;
      xh[(size_t)r * K + v] = -box + (std::cos(M_PI * (double)d / (double)(nnodes - 1)) + 1.0) * box;
    }
  }
  const int rc = os_kl_model_finish(md, K, xh, mu, modes, (hipStream_t)stream, "kl_interp_os_build");
  if (rc == STOMSFEM_OK) *model = md;
  return rc;
}

int stomsfem_kl_sgi_os_build(int32_t ncx, int32_t ncy, int32_t m, int32_t oversample, int32_t K, const double* mu,
                             const double* modes, int32_t level, double box, stomsfem_model** model, void* stream) {
  if (!model) return fail(STOMSFEM_EINVAL, "kl_sgi_os_build: NULL model");
  *model = nullptr;
  const int o = oversample, P = m + 2 * oversample;
  if (ncx < 1 || ncx != ncy || m < 1 || o < 1 || o > m || !upscale_os_supports(m, o) || P > ncx * m || K < 1 ||
      K > RI_KMAX || level < 0 || level > SGI_LEVEL_MAX || !(box > 0))
    return fail(STOMSFEM_EINVAL,
                "kl_sgi_os_build: need a square mesh, 1 <= oversample <= m, m + 2 oversample <= 64 and <= the "
                "domain, 1 <= K <= 4, 0 <= level <= 5, box > 0");
  if (!device_ptr(mu) || !device_ptr(modes)) return fail(STOMSFEM_EINVAL, "kl_sgi_os_build: mu and modes on device");
  if (ncx * ncy > 65535) return fail(STOMSFEM_EINVAL, "kl_sgi_os_build: at most 65535 coarse elements");
  SgiComb C;
  sgi_combination(level, C);
  if (C.missing) return fail(STOMSFEM_EINVAL, "kl_sgi_os_build: a tensor node of the combination is not a grid node");
  const int64_t rows = C.npts[K];
  auto* md = os_kl_model(8, ncx, ncy, m, o, box, rows);
  md->sc_level = level;
  md->sg_nb = (int32_t)C.nodes.size();
  md->sg_kmax = K;
  std::memcpy(md->sg_lofs, C.lofs, sizeof(C.lofs));
  std::memcpy(md->sg_rofs, C.rofs, sizeof(C.rofs));
  hipError_t e = hipMalloc((void**)&md->cb_coef, sizeof(double) * C.cc.size());
  if (e == hipSuccess) e = hipMalloc((void**)&md->cb_boff, sizeof(uint32_t) * C.cbo.size());
  if (e == hipSuccess) e = hipMalloc((void**)&md->cb_rows, sizeof(int32_t) * C.rows_all.size());
  if (e == hipSuccess) e = hipMalloc((void**)&md->sg_nodes, sizeof(double) * C.nodes.size());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    model_release(md);
    return fail(STOMSFEM_ENOMEM, "kl_sgi_os_build: device allocation failed");
  }
  e = hipMemcpy(md->cb_coef, C.cc.data(), sizeof(double) * C.cc.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(md->cb_boff, C.cbo.data(), sizeof(uint32_t) * C.cbo.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(md->cb_rows, C.rows_all.data(), sizeof(int32_t) * C.rows_all.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(md->sg_nodes, C.nodes.data(), sizeof(double) * C.nodes.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    model_release(md);
    return hip_fail(e, "kl_sgi_os_build");
  }
  // grid nodes: Chebyshev-Lobatto points of the finest level, by digit
  std::vector<double> xh((size_t)rows * K);
  for (int64_t r = 0; r < rows; ++r)
    for (int v = 0; v < K; ++v) {
      const int32_t c = C.gdig[K][r * K + v];
      xh[(size_t)r * K + v] = -box + (std::cos(M_PI * (double)c / (double)C.D) + 1.0) * box;
    }
  const int rc = os_kl_model_finish(md, K, xh, mu, modes, (hipStream_t)stream, "kl_sgi_os_build");
  if (rc == STOMSFEM_OK) *model = md;
  return rc;
}

int stomsfem_kl_interp_apply(stomsfem_model* model, const double* xi, const double* kappa, int64_t nsamples,
                             double* S, int32_t* status, int64_t* nfallback, void* stream) {
  if (nfallback) *nfallback = 0;
  if (!model || (model->kind != 6 && model->kind != 7 && model->kind != 8))
    return fail(STOMSFEM_EINVAL, "kl_interp_apply: not a KL interpolation model");
  const bool os = model->kind == 7 || model->kind == 8;
  if (nsamples < 0) return fail(STOMSFEM_EINVAL, "kl_interp_apply: nsamples < 0");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(xi) || !device_ptr(kappa) || !device_ptr(S) || (status && !device_ptr(status)))
    return fail(STOMSFEM_EINVAL, "kl_interp_apply: arrays must be device pointers");
  const int Mc = model->ncx * model->ncy, K = model->lv_max;
  hipStream_t st = (hipStream_t)stream;
  OrderedUse order;  // the model's scratch buffers
  if (int orc = order.begin(model->order_mu, model->order_ev, st); orc != STOMSFEM_OK) return orc;
  const int64_t need = nsamples * Mc;
  if (model->list_cap < need) {
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
      hipFree(model->list);
      model->list = nullptr;
      model->list_cap = 0;
      e = hipMalloc(&model->list, sizeof(int64_t) * need);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(STOMSFEM_ENOMEM, "kl_interp_apply: fallback list allocation failed");
    }
    model->list_cap = need;
  }
  RiApplyArgs a{};
  a.npatch = Mc;
  a.nxi = Mc * K;
  a.nn = model->nn;
  a.ne = os ? 16 : 10;
  a.nsamples = nsamples;
  a.lo = model->lo;
  a.hi = model->hi;
  a.table = model->table;
  a.off = model->off;
  a.lv = model->lv;
  a.nlv = model->nlv;
  a.xi = xi;
  a.S = S;
  a.status = status;
  a.list = model->list;
  a.list_count = model->counter;
  hipError_t e = launch_zero_u64(model->counter, st);
  if (e == hipSuccess && model->kind == 8) {
    // Smolyak interpolant on the sparse grid (every element has K variables)
    SgiApplyArgs g{};
    g.ne = 16;
    g.npatch = Mc;
    g.nxi = Mc * K;
    g.level = model->sc_level;
    g.nb = model->sg_nb;
    g.kmax = model->sg_kmax;
    g.nsamples = nsamples;
    g.lo = model->lo;
    g.hi = model->hi;
    g.table = model->table;
    g.off = model->off;
    g.lv = model->lv;
    g.nlv = model->nlv;
    g.nodes = model->sg_nodes;
    std::memcpy(g.lofs, model->sg_lofs, sizeof(g.lofs));
    std::memcpy(g.rofs, model->sg_rofs, sizeof(g.rofs));
    g.cb_coef = model->cb_coef;
    g.cb_boff = model->cb_boff;
    g.cb_rows = model->cb_rows;
    g.xi = xi;
    g.S = S;
    g.status = status;
    g.list = model->list;
    g.list_count = model->counter;
    e = launch_sgi_apply(g, st);
  } else if (e == hipSuccess) {
    e = launch_ri_apply(a, st);
  }
  unsigned long long n = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&n, model->counter, sizeof(n), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "kl_interp_apply");
  if (n > (unsigned long long)need) return fail(STOMSFEM_EHIP, "kl_interp_apply: fallback count out of range");
  if (nfallback) *nfallback = (int64_t)n;
  if (os) {
    // out-of-box pairs: the oversampling kernels on the sample's own field,
    // for the listed pairs only
    UpArgs full{};
    full.nsamples = nsamples;
    full.ncx = model->ncx;
    full.ncy = model->ncy;
    full.m = model->m;
    full.npairs = nsamples * Mc;
    full.a = kappa;
    full.S = model->Sc;
    full.status = model->stc;
    // Sc, stc hold chunk 3 x 3 meshes of the build: 9 chunk pairs here (one
    // launch for all of them is what matters: each pair is a long dependent
    // elimination, so launches in sequence add their latencies)
    const int64_t fchunk = 9 * model->chunk;
    for (int64_t start = 0; start < (int64_t)n; start += fchunk) {
      const int64_t cnt = std::min<int64_t>(fchunk, (int64_t)n - start);
      e = launch_upscale_os(full, model->os_o, STOMSFEM_F64, st, model->list + start, cnt);
      if (e == hipSuccess)
        e = launch_scatter_pairs(model->list + start, cnt, model->Sc, model->stc, S, status, 1, st, 16);
      if (e != hipSuccess) return hip_fail(e, "kl_interp_apply: oversampled solve launch");
    }
    return STOMSFEM_OK;
  }
  // out-of-box pairs: the plain path on the sample's own coefficient block
  UpArgs full{};
  full.nsamples = nsamples;
  full.ncx = model->ncx;
  full.ncy = model->ncy;
  full.m = model->m;
  full.a = kappa;
  for (int64_t start = 0; start < (int64_t)n; start += model->chunk) {
    const int64_t cnt = std::min<int64_t>(model->chunk, (int64_t)n - start);
    e = launch_gather_blocks(full, STOMSFEM_F64, model->list + start, cnt, model->blk, st);
    if (e == hipSuccess) {
      UpArgs u{};
      u.nsamples = cnt;
      u.ncx = u.ncy = 1;
      u.m = model->m;
      u.npairs = cnt;
      u.a = model->blk;
      u.S = model->Sc;
      u.status = model->stc;
      e = launch_upscale_any(u, STOMSFEM_F64, st);
    }
    if (e == hipSuccess) e = launch_scatter_pairs(model->list + start, cnt, model->Sc, model->stc, S, status, 1, st);
    if (e != hipSuccess) return hip_fail(e, "kl_interp_apply: plain solve launch");
  }
  return STOMSFEM_OK;
}

int stomsfem_upscale_os(const stomsfem_batch* batch, int32_t oversample, void* stream) {
  if (!batch) return fail(STOMSFEM_EINVAL, "upscale_os: NULL batch");
  int rc = check_batch(*batch, 0);
  if (rc != STOMSFEM_OK) return rc;
  const stomsfem_batch& b = *batch;
  if (oversample < 0 || !upscale_os_supports(b.m, oversample))
    return fail(STOMSFEM_EINVAL, "upscale_os: need oversample >= 0 and 2 <= m + 2*oversample <= 64");
  const int64_t M = b.m + 2 * (int64_t)oversample;
  if (M > (int64_t)b.ncx * b.m || M > (int64_t)b.ncy * b.m)
    return fail(STOMSFEM_EINVAL, "upscale_os: the oversampled patch is larger than the domain");
  if (b.nsamples == 0) return STOMSFEM_OK;
  hipError_t e = launch_upscale_os(to_args(b), oversample, b.a_dtype, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "upscale_os launch");
}

int stomsfem_coarse_solve_pg(int32_t ncx, int32_t ncy, int64_t nsamples, const double* S16, const double* load,
                             double* U, double* qoi_mean, double* qoi_var, int32_t* status, void* stream) {
  if (ncx < 1 || ncy < 1 || nsamples < 0) return fail(STOMSFEM_EINVAL, "coarse_solve_pg: bad sizes");
  if (ncx > 64 || ncy > 1024) return fail(STOMSFEM_EINVAL, "coarse_solve_pg: need ncx <= 64 and ncy <= 1024");
  if (coarse_lds_bytes(ncx, true) > 64 * 1024)
    return fail(STOMSFEM_EINVAL, "coarse_solve_pg: ncx too large for the LDS window");
  const int nU = (ncx - 1) * (ncy - 1);
  if (nU == 0) return STOMSFEM_OK;
  if (nsamples > 0 && (!device_ptr(S16) || !device_ptr(U)))
    return fail(STOMSFEM_EINVAL, "coarse_solve_pg: S16 and U must be device pointers");
  if (load && !device_ptr(load)) return fail(STOMSFEM_EINVAL, "coarse_solve_pg: load must be a device pointer");
  if ((qoi_mean && !device_ptr(qoi_mean)) || (qoi_var && !device_ptr(qoi_var)))
    return fail(STOMSFEM_EINVAL, "coarse_solve_pg: qoi outputs must be device pointers");
  if (status && !device_ptr(status)) return fail(STOMSFEM_EINVAL, "coarse_solve_pg: status must be a device pointer");
  void* work = nullptr;
  WorkspaceLease lease;
  if (nsamples > 0) {
    int rc = lease.acquire(sizeof(double) * (size_t)coarse_work_doubles(ncx, ncy, nsamples), (hipStream_t)stream,
                           &work);
    if (rc != STOMSFEM_OK) return rc;
  }
  hipError_t e = launch_coarse_pg(ncx, ncy, nsamples, S16, load, U, qoi_mean, qoi_var, status, (double*)work,
                                  (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "coarse_solve_pg launch");
}

namespace {
// The reduced-basis build; m_max = 48 for stomsfem_reduce (the batch limit),
// 64 for the oversampled patches (cells past 32 take the band-window snapshot
// kernel).
int reduce_build(const stomsfem_batch* train, int32_t r_max, double tail_tol, stomsfem_model** model, void* stream,
                 int m_max) {
  if (!train || !model) return fail(STOMSFEM_EINVAL, "reduce: NULL argument");
  *model = nullptr;
  const stomsfem_batch& b = *train;
  if (b.ncx < 1 || b.ncy < 1 || b.m < 2 || b.m > m_max)
    return fail(STOMSFEM_EINVAL, "reduce: need 2 <= m <= " + std::to_string(m_max));
  if (b.a_dtype != STOMSFEM_F64 && b.a_dtype != STOMSFEM_F32) return fail(STOMSFEM_EINVAL, "reduce: bad a_dtype");
  if (b.nsamples < 1) return fail(STOMSFEM_EINVAL, "reduce: need at least one training sample");
  if (r_max < 1 || r_max > 8) return fail(STOMSFEM_EINVAL, "reduce: r_max must be in 1..8");
  if (!(tail_tol >= 0.0)) return fail(STOMSFEM_EINVAL, "reduce: tail_tol must be >= 0");
  if (!device_ptr(b.a)) return fail(STOMSFEM_EINVAL, "reduce: a is not a device pointer");
  const int m = b.m, nI = (m - 1) * (m - 1), Mc = b.ncx * b.ncy;
  if (b.nsamples > 341 || (!rb_dual(m, (int)b.nsamples) && nI > 1024))
    return fail(STOMSFEM_EINVAL, "reduce: the eigenproblem (the smaller of (m-1)^2 and 3 ntrain) must be <= 1024, "
                                 "and ntrain <= 341");
  if (b.nsamples * (int64_t)Mc > (int64_t{1} << 31))
    return fail(STOMSFEM_EINVAL, "reduce: too many training pairs");
  hipStream_t st = (hipStream_t)stream;
  auto* md = new stomsfem_model();
  md->kind = 1;
  hipGetDevice(&md->device);
  md->ncx = b.ncx;
  md->ncy = b.ncy;
  md->m = m;
  md->rmax = 8;
  md->KD = rb_pad_kd(m);
  md->PP = rb_pad_p(md->rmax);
  double* phi = nullptr;
  double* work = nullptr;
  hipError_t e = hipSuccess;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  };
  A((void**)&md->rK, sizeof(int32_t) * Mc);
  A((void**)&md->lambda, sizeof(double) * Mc * nI);
  A((void**)&md->Z, sizeof(double) * (size_t)Mc * nI * md->rmax);
  A((void**)&md->phibar, sizeof(double) * (size_t)Mc * 3 * nI);
  A((void**)&md->G32, sizeof(float) * (size_t)Mc * md->KD * md->PP);
  A((void**)&md->G64, sizeof(double) * (size_t)Mc * md->KD * md->PP);
  A((void**)&phi, sizeof(double) * (size_t)b.nsamples * Mc * 3 * nI);
  A((void**)&work, sizeof(double) * (size_t)rb_work_doubles(b.ncx, b.ncy, m, (int)b.nsamples));
  // snapshots: the FP64 band in LDS where it fits (m <= 26), the FP64
  // band-window kernel (global row store) beyond
  const bool band_phi = cell_phi_lds_bytes(m) > CELL_PHI_LDS_MAX;
  const int64_t band_blocks = band_phi ? std::min<int64_t>(b.nsamples * Mc, 1024) : 0;
  double* band_ws = nullptr;
  if (band_phi) A((void**)&band_ws, sizeof(double) * (size_t)band_blocks * cell_phi_band_ws_doubles(m));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    hipFree(phi);
    hipFree(work);
    hipFree(band_ws);
    model_release(md);
    return fail(STOMSFEM_ENOMEM, "reduce: device allocation failed");
  }
  UpArgs up = to_args(b);
  up.S = nullptr;
  up.status = nullptr;
  if (band_phi)
    e = launch_cell_phi_band(up, b.a_dtype, phi, band_ws, band_blocks, st);
  else
    e = launch_cell_phi(up, b.a_dtype, phi, st);
  if (e == hipSuccess) {
    RbBuildArgs ba{};
    ba.ncx = b.ncx;
    ba.ncy = b.ncy;
    ba.m = m;
    ba.ntrain = (int32_t)b.nsamples;
    ba.rmax = md->rmax;
    ba.rcap = r_max;
    ba.tail_tol = tail_tol;
    ba.a = b.a;
    ba.a_dtype = b.a_dtype;
    ba.phi = phi;
    ba.work = work;
    ba.Z = md->Z;
    ba.phibar = md->phibar;
    ba.lambda = md->lambda;
    ba.rK = md->rK;
    ba.G32 = md->G32;
    ba.G64 = md->G64;
    ba.KD = md->KD;
    ba.PP = md->PP;
    ba.max_sweeps = 30;
    e = launch_rb_build(ba, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(phi);
  hipFree(work);
  hipFree(band_ws);
  if (e != hipSuccess) {
    model_release(md);
    return hip_fail(e, "reduce");
  }
  *model = md;
  return STOMSFEM_OK;
}
}  // namespace

int stomsfem_reduce(const stomsfem_batch* train, int32_t r_max, double tail_tol, stomsfem_model** model,
                    void* stream) {
  return reduce_build(train, r_max, tail_tol, model, stream, 48);
}

int stomsfem_reduce_apply(const stomsfem_model* model, const stomsfem_batch* batch, int32_t precision,
                          void* stream) {
  if (!model || !batch) return fail(STOMSFEM_EINVAL, "reduce_apply: NULL argument");
  if (model->kind != 1) return fail(STOMSFEM_EINVAL, "reduce_apply: not a reduced-basis model");
  int rc = check_batch(*batch, 0);
  if (rc != STOMSFEM_OK) return rc;
  if (batch->ncx != model->ncx || batch->ncy != model->ncy || batch->m != model->m)
    return fail(STOMSFEM_EINVAL, "reduce_apply: batch mesh differs from the model's");
  if (precision != STOMSFEM_PREC_F64 && precision != STOMSFEM_PREC_F32)
    return fail(STOMSFEM_EINVAL, "reduce_apply: precision must be STOMSFEM_PREC_F64 or STOMSFEM_PREC_F32");
  const bool f64 = precision == STOMSFEM_PREC_F64;
  if (!f64 && (model->KD % 64 != 0 || model->PP != 80))
    return fail(STOMSFEM_EINVAL, "reduce_apply: the model's table layout does not serve the MFMA stage (FP64 only)");
  if (batch->nsamples == 0) return STOMSFEM_OK;
  RbApplyArgs ra{};
  ra.up = to_args(*batch);
  ra.rmax = model->rmax;
  ra.KD = model->KD;
  ra.PP = model->PP;
  ra.rK = model->rK;
  ra.G32 = model->G32;
  ra.G64 = model->G64;
  hipError_t e = launch_rb_apply(ra, batch->a_dtype, f64, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "reduce_apply launch");
}

int stomsfem_reduce_os(const stomsfem_batch* train, int32_t oversample, int32_t r_max, double tail_tol,
                       stomsfem_model** model, void* stream) {
  if (!train || !model) return fail(STOMSFEM_EINVAL, "reduce_os: NULL argument");
  *model = nullptr;
  const stomsfem_batch& b = *train;
  if (b.ncx < 1 || b.ncy < 1 || b.m < 1 || oversample < 0)
    return fail(STOMSFEM_EINVAL, "reduce_os: need ncx, ncy, m >= 1 and oversample >= 0");
  const int Mp = b.m + 2 * oversample;
  if (Mp < 2 || Mp > 64) return fail(STOMSFEM_EINVAL, "reduce_os: need 2 <= m + 2*oversample <= 64");
  if (Mp > b.ncx * b.m || Mp > b.ncy * b.m)
    return fail(STOMSFEM_EINVAL, "reduce_os: the patch is larger than the domain");
  if (b.a_dtype != STOMSFEM_F64 && b.a_dtype != STOMSFEM_F32)
    return fail(STOMSFEM_EINVAL, "reduce_os: bad a_dtype");
  if (b.nsamples < 1) return fail(STOMSFEM_EINVAL, "reduce_os: need at least one training sample");
  if (b.nsamples > 341) return fail(STOMSFEM_EINVAL, "reduce_os: ntrain must be <= 341");
  if (!device_ptr(b.a)) return fail(STOMSFEM_EINVAL, "reduce_os: a is not a device pointer");
  hipStream_t st = (hipStream_t)stream;
  const int64_t nemb = b.nsamples * (int64_t)b.ncy * Mp * b.ncx * Mp;
  double* emb = nullptr;
  hipError_t e = hipMalloc((void**)&emb, sizeof(double) * nemb);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(STOMSFEM_ENOMEM, "reduce_os: device allocation failed");
  }
  e = launch_rb_os_embed(b.a, b.a_dtype, b.nsamples, b.ncx, b.ncy, b.m, oversample, emb, st);
  if (e != hipSuccess) {
    hipFree(emb);
    return hip_fail(e, "reduce_os: gather of the patches");
  }
  // the patches as the elements of a batch of side Mp
  stomsfem_batch pb = b;
  pb.m = Mp;
  pb.a = emb;
  pb.a_dtype = STOMSFEM_F64;
  pb.S = nullptr;
  pb.status = nullptr;
  stomsfem_model* md = nullptr;
  int rc = reduce_build(&pb, r_max, tail_tol, &md, stream, 64);
  hipStreamSynchronize(st);
  hipFree(emb);
  if (rc != STOMSFEM_OK) return rc;
  md->kind = 9;
  md->os_o = oversample;
  md->os_m = b.m;
  const int Mc = b.ncx * b.ncy;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  };
  A((void**)&md->GO, sizeof(double) * (size_t)Mc * md->KD * RBO_PO);
  A((void**)&md->GO32, sizeof(float) * (size_t)Mc * md->KD * RBO_PO);
  A((void**)&md->Pc, sizeof(double) * (size_t)Mc * 4 * RBO_NF);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    model_release(md);
    return fail(STOMSFEM_ENOMEM, "reduce_os: device allocation failed");
  }
  RbOsArgs t = rb_os_args(md);
  e = launch_rb_os_tables(t, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    model_release(md);
    return hip_fail(e, "reduce_os: online tables");
  }
  // the plain patch tables are not used online
  hipFree(md->G32);
  hipFree(md->G64);
  md->G32 = nullptr;
  md->G64 = nullptr;
  *model = md;
  return STOMSFEM_OK;
}

int stomsfem_reduce_os_apply(const stomsfem_model* model, const stomsfem_batch* batch, int32_t precision,
                             void* stream) {
  if (!model || !batch) return fail(STOMSFEM_EINVAL, "reduce_os_apply: NULL argument");
  if (model->kind != 9) return fail(STOMSFEM_EINVAL, "reduce_os_apply: not a model of stomsfem_reduce_os");
  int rc = check_batch(*batch, 0);
  if (rc != STOMSFEM_OK) return rc;
  if (batch->ncx != model->ncx || batch->ncy != model->ncy || batch->m != model->os_m)
    return fail(STOMSFEM_EINVAL, "reduce_os_apply: batch mesh differs from the model's");
  if (precision != STOMSFEM_PREC_F64 && precision != STOMSFEM_PREC_F32)
    return fail(STOMSFEM_EINVAL, "reduce_os_apply: precision must be STOMSFEM_PREC_F64 or STOMSFEM_PREC_F32");
  if (batch->nsamples == 0) return STOMSFEM_OK;
  hipError_t e = hipSuccess;
  if (precision == STOMSFEM_PREC_F64) {
    e = launch_rb_os_apply(rb_os_args(model), to_args(*batch), batch->a_dtype, (hipStream_t)stream);
  } else {
    RbApplyArgs ra{};
    ra.up = to_args(*batch);
    ra.rmax = model->rmax;
    ra.KD = model->KD;
    ra.PP = RBO_PO;
    ra.rK = model->rK;
    ra.G32 = model->GO32;
    ra.os_o = model->os_o;
    ra.Pc = model->Pc;
    e = launch_rb_os_apply_mfma(ra, batch->a_dtype, (hipStream_t)stream);
  }
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "reduce_os_apply launch");
}

int stomsfem_model_export(const stomsfem_model* model, int32_t which, void* host_dst, int64_t bytes) {
  if (!model || !host_dst) return fail(STOMSFEM_EINVAL, "model_export: NULL argument");
  const int Mc = model->ncx * model->ncy, nI = (model->m - 1) * (model->m - 1);
  const void* src = nullptr;
  int64_t need = 0;
  if (which >= 0 && which <= 3 && model->kind != 1 && model->kind != 9)
    return fail(STOMSFEM_EINVAL, "model_export: not a reduced-basis model");
  switch (which) {
    case 0: src = model->rK; need = 4LL * Mc; break;
    case 1: src = model->lambda; need = 8LL * Mc * nI; break;
    case 2: src = model->Z; need = 8LL * Mc * nI * model->rmax; break;
    case 3: src = model->phibar; need = 8LL * Mc * 3 * nI; break;
    case 4:
      if (model->kind != 3) return fail(STOMSFEM_EINVAL, "model_export: not an interpolation model");
      src = model->table; need = 8LL * model->rows * 10; break;
    case 5:
      if (model->kind != 3) return fail(STOMSFEM_EINVAL, "model_export: not an interpolation model");
      src = model->off; need = 8LL * (Mc + 1); break;
    default: return fail(STOMSFEM_EINVAL, "model_export: unknown array");
  }
  if (bytes != need) return fail(STOMSFEM_EINVAL, "model_export: size mismatch, expected " + std::to_string(need));
  hipError_t e = hipMemcpy(host_dst, src, (size_t)need, hipMemcpyDeviceToHost);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "model_export");
}

int stomsfem_model_free(stomsfem_model* model) {
  model_release(model);
  return STOMSFEM_OK;
}

// ---------------------------------------------------------------------------
// learned surrogate
// ---------------------------------------------------------------------------
int stomsfem_local_vars_bumps(int32_t ncx, int32_t ncy, int32_t m, const stomsfem_bump_family* fam, int32_t kmax,
                              int32_t* local_vars, int32_t* nlocal) {
  if (!fam || !local_vars || ncx < 1 || ncy < 1 || m < 1 || kmax < 1 || fam->g < 1 || !(fam->rho > 0))
    return fail(STOMSFEM_EINVAL, "local_vars_bumps: bad arguments");
  const int nfx = ncx * m;  // square fine cells of side 1 / (ncx m)
  const double h = 1.0 / nfx;
  for (int K = 0; K < ncx * ncy; ++K) {
    const int kx = K % ncx, ky = K / ncx;
    int cnt = 0;
    for (int j = 0; j < fam->g * fam->g; ++j) {
      const double cx = ((j % fam->g) + 0.5) / fam->g, cy = ((j / fam->g) + 0.5) / fam->g;
      bool touch = false;
      for (int ey = 0; ey < m && !touch; ++ey)
        for (int ex = 0; ex < m && !touch; ++ex) {
          const double x = (kx * m + ex + 0.5) * h, y = (ky * m + ey + 0.5) * h;
          const double r2 = ((x - cx) * (x - cx) + (y - cy) * (y - cy)) / (fam->rho * fam->rho);
          touch = r2 < 1.0;
        }
      if (!touch) continue;
      if (cnt >= kmax) return fail(STOMSFEM_EINVAL, "local_vars_bumps: more than kmax local variables");
      local_vars[K * kmax + cnt++] = j;
    }
    for (int c = cnt; c < kmax; ++c) local_vars[K * kmax + c] = -1;
    if (nlocal) nlocal[K] = cnt;
  }
  return STOMSFEM_OK;
}

int stomsfem_local_vars_features(int32_t ncx, int32_t ncy, int32_t m, const int32_t* map, int32_t nfeat,
                                 int32_t kmax, int32_t* local_vars, int32_t* nlocal) {
  if (!map || !local_vars) return fail(STOMSFEM_EINVAL, "local_vars_features: NULL argument");
  if (ncx < 1 || ncy < 1 || m < 1 || nfeat < 1 || kmax < 1)
    return fail(STOMSFEM_EINVAL, "local_vars_features: bad sizes");
  const int64_t nfx = (int64_t)ncx * m;
  for (int K = 0; K < ncx * ncy; ++K) {
    const int kx = K % ncx, ky = K / ncx;
    std::vector<int32_t> feats;
    for (int ey = 0; ey < m; ++ey)
      for (int ex = 0; ex < m; ++ex) {
        const int32_t f = map[(int64_t)(ky * m + ey) * nfx + kx * m + ex];
        if (f < -1 || f >= nfeat) return fail(STOMSFEM_EINVAL, "local_vars_features: map entry out of range");
        if (f >= 0) feats.push_back(f);
      }
    std::sort(feats.begin(), feats.end());
    feats.erase(std::unique(feats.begin(), feats.end()), feats.end());
    const int cnt = (int)feats.size();
    for (int c = 0; c < kmax; ++c)
      local_vars[K * kmax + c] = cnt > kmax ? (c == 0 ? MLP_LV_ALWAYS_PLAIN : -1) : (c < cnt ? feats[c] : -1);
    if (nlocal) nlocal[K] = cnt;
  }
  return STOMSFEM_OK;
}

static int mlp_create_common(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars, const float* init_params,
                             const stomsfem_bump_family* fam, double box, stomsfem_model** model);

int stomsfem_mlp_create_features(int32_t nc, int32_t m, const int32_t* map, int32_t nfeat, double decades,
                                 const float* init_params, double box, stomsfem_model** model) {
  if (!map || !init_params || !model) return fail(STOMSFEM_EINVAL, "mlp_create_features: NULL argument");
  if (nc < 1 || m < 1 || m > 48 || nfeat < 1) return fail(STOMSFEM_EINVAL, "mlp_create_features: bad sizes");
  if (!(decades > 0) || !(box > 0)) return fail(STOMSFEM_EINVAL, "mlp_create_features: need decades > 0 and box > 0");
  if (!device_ptr(map)) return fail(STOMSFEM_EINVAL, "mlp_create_features: map must be a device pointer");
  *model = nullptr;
  const int64_t nf = (int64_t)nc * m;
  std::vector<int32_t> hmap((size_t)(nf * nf));
  hipError_t e = hipMemcpy(hmap.data(), map, sizeof(int32_t) * hmap.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "mlp_create_features");
  const int Mc = nc * nc;
  std::vector<int32_t> lv((size_t)Mc * MLP_KIN);
  int rc = stomsfem_local_vars_features(nc, nc, m, hmap.data(), nfeat, MLP_KIN, lv.data(), nullptr);
  if (rc != STOMSFEM_OK) return rc;
  // fraction of each patch's boundary ring of fine elements owned by each
  // local feature (the output scale of the network)
  std::vector<double> rw((size_t)Mc * MLP_KIN, 0.0);
  const int nring = m == 1 ? 1 : 4 * m - 4;
  for (int K = 0; K < Mc; ++K) {
    const int kx = K % nc, ky = K / nc;
    for (int ey = 0; ey < m; ++ey)
      for (int ex = 0; ex < m; ++ex) {
        if (ey != 0 && ey != m - 1 && ex != 0 && ex != m - 1) continue;
        const int32_t f = hmap[(int64_t)(ky * m + ey) * nf + kx * m + ex];
        for (int c = 0; c < MLP_KIN; ++c)
          if (f >= 0 && lv[K * MLP_KIN + c] == f) rw[K * MLP_KIN + c] += 1.0 / nring;
      }
  }
  stomsfem_model* md = nullptr;
  rc = mlp_create_common(nc, nc, m, lv.data(), init_params, nullptr, box, &md);
  if (rc != STOMSFEM_OK) return rc;
  md->family = MLP_FAMILY_FEATURES;
  md->nfeat = nfeat;
  md->decades = decades;
  md->lv_max = std::max(md->lv_max, nfeat - 1);
  e = hipMalloc(&md->fmap, sizeof(int32_t) * hmap.size());
  if (e == hipSuccess) e = hipMemcpy(md->fmap, hmap.data(), sizeof(int32_t) * hmap.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&md->rw, sizeof(double) * rw.size());
  if (e == hipSuccess) e = hipMemcpy(md->rw, rw.data(), sizeof(double) * rw.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !md->blk) {  // the chunked plain fallback serves every m for this family
    md->chunk = std::max<int64_t>(256, std::min<int64_t>(65536, (int64_t{1} << 25) / ((int64_t)m * m)));
    e = hipMalloc(&md->blk, sizeof(double) * (size_t)md->chunk * m * m);
    if (e == hipSuccess) e = hipMalloc(&md->Sc, sizeof(double) * (size_t)md->chunk * 10);
    if (e == hipSuccess) e = hipMalloc(&md->stc, sizeof(int32_t) * (size_t)md->chunk);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    model_release(md);
    return fail(STOMSFEM_ENOMEM, "mlp_create_features: device allocation failed");
  }
  *model = md;
  return STOMSFEM_OK;
}

int stomsfem_mlp_create(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars, const float* init_params,
                        const stomsfem_bump_family* fam, double box, stomsfem_model** model) {
  return mlp_create_common(ncx, ncy, m, local_vars, init_params, fam, box, model);
}

static int mlp_create_common(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars, const float* init_params,
                             const stomsfem_bump_family* fam, double box, stomsfem_model** model) {
  if (!local_vars || !init_params || !model) return fail(STOMSFEM_EINVAL, "mlp_create: NULL argument");
  if (ncx < 1 || ncy < 1 || m < 1 || m > 48) return fail(STOMSFEM_EINVAL, "mlp_create: need 1 <= m <= 48");
  if (!(box > 0)) return fail(STOMSFEM_EINVAL, "mlp_create: box must be > 0");
  *model = nullptr;
  const int Mc = ncx * ncy;
  auto* md = new stomsfem_model();
  md->kind = 2;
  hipGetDevice(&md->device);
  md->ncx = ncx;
  md->ncy = ncy;
  md->m = m;
  md->box = box;
  if (fam) md->fam = *fam;
  for (int i = 0; i < Mc * MLP_KIN; ++i) {
    if (local_vars[i] < -1 && !(local_vars[i] == MLP_LV_ALWAYS_PLAIN && i % MLP_KIN == 0)) {
      delete md;
      return fail(STOMSFEM_EINVAL, "mlp_create: local variable indices must be >= 0 or -1 (padding)");
    }
    if (local_vars[i] > md->lv_max) md->lv_max = local_vars[i];
  }
  hipError_t e = hipSuccess;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  };
  A((void**)&md->lv, sizeof(int32_t) * Mc * MLP_KIN);
  A((void**)&md->params, sizeof(float) * (size_t)Mc * MLP_NP);
  A((void**)&md->m1, sizeof(float) * (size_t)Mc * MLP_NP);
  A((void**)&md->m2, sizeof(float) * (size_t)Mc * MLP_NP);
  A((void**)&md->mu, sizeof(double) * Mc * 10);
  A((void**)&md->sd, sizeof(double) * Mc * 10);
  A((void**)&md->sd_raw, sizeof(double) * Mc * 10);
  A((void**)&md->counter, sizeof(unsigned long long));
  if (m != 8) {  // buffers of the chunked plain fallback (regenerate, upscale, compare)
    md->chunk = std::max<int64_t>(256, std::min<int64_t>(65536, (int64_t{1} << 25) / ((int64_t)m * m)));
    A((void**)&md->blk, sizeof(double) * (size_t)md->chunk * m * m);
    A((void**)&md->Sc, sizeof(double) * (size_t)md->chunk * 10);
    A((void**)&md->stc, sizeof(int32_t) * (size_t)md->chunk);
  }
  if (e == hipSuccess) e = hipMemcpy(md->lv, local_vars, sizeof(int32_t) * Mc * MLP_KIN, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->params, init_params, sizeof(float) * (size_t)Mc * MLP_NP, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(md->m1, 0, sizeof(float) * (size_t)Mc * MLP_NP);
  if (e == hipSuccess) e = hipMemset(md->m2, 0, sizeof(float) * (size_t)Mc * MLP_NP);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    model_release(md);
    return fail(STOMSFEM_ENOMEM, "mlp_create: device allocation failed");
  }
  *model = md;
  return STOMSFEM_OK;
}

int stomsfem_mlp_set_data(stomsfem_model* model, const double* xi, int32_t nxi, const double* S, int64_t ntrain,
                          void* stream) {
  if (!model || model->kind != 2) return fail(STOMSFEM_EINVAL, "mlp_set_data: not a surrogate model");
  if (ntrain < 1 || nxi < 1) return fail(STOMSFEM_EINVAL, "mlp_set_data: bad sizes");
  if (model->lv_max >= nxi) return fail(STOMSFEM_EINVAL, "mlp_set_data: nxi smaller than the local variable indices");
  if (!device_ptr(xi) || !device_ptr(S)) return fail(STOMSFEM_EINVAL, "mlp_set_data: xi and S must be device pointers");
  const int Mc = model->ncx * model->ncy;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "mlp_set_data");
  hipFree(model->X);
  hipFree(model->T);
  model->X = model->T = nullptr;
  e = hipMalloc(&model->X, sizeof(float) * (size_t)Mc * ntrain * MLP_KIN);
  if (e == hipSuccess) e = hipMalloc(&model->T, sizeof(float) * (size_t)Mc * ntrain * 10);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(STOMSFEM_ENOMEM, "mlp_set_data: device allocation failed");
  }
  model->ntrain = ntrain;
  MlpDataArgs d{};
  d.family = model->family;
  d.decades = model->decades;
  d.rw = model->rw;
  d.npatch = Mc;
  d.nxi = nxi;
  d.ntrain = ntrain;
  d.lv = model->lv;
  d.xi = xi;
  d.S = S;
  d.mu = model->mu;
  d.sd = model->sd;
  d.sd_raw = model->sd_raw;
  d.X = model->X;
  d.T = model->T;
  e = launch_mlp_data(d, st);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "mlp_set_data launch");
}

int stomsfem_mlp_train(stomsfem_model* model, int32_t steps, float lr, const int64_t* perm, float* loss, void* stream) {
  if (!model || model->kind != 2) return fail(STOMSFEM_EINVAL, "mlp_train: not a surrogate model");
  if (model->ntrain < 1) return fail(STOMSFEM_EINVAL, "mlp_train: no training data (stomsfem_mlp_set_data)");
  if (steps < 0 || !(lr > 0)) return fail(STOMSFEM_EINVAL, "mlp_train: bad steps or lr");
  if (perm && !device_ptr(perm)) return fail(STOMSFEM_EINVAL, "mlp_train: perm must be a device pointer");
  if (loss && !device_ptr(loss)) return fail(STOMSFEM_EINVAL, "mlp_train: loss must be a device pointer");
  if (steps == 0) return STOMSFEM_OK;
  OrderedUse order;  // parameters and moments
  if (int orc = order.begin(model->order_mu, model->order_ev, (hipStream_t)stream); orc != STOMSFEM_OK) return orc;
  MlpTrainArgs t{};
  t.npatch = model->ncx * model->ncy;
  t.ntrain = model->ntrain;
  t.steps = steps;
  t.t0 = model->adam_t;
  t.lr = lr;
  t.params = model->params;
  t.m1 = model->m1;
  t.m2 = model->m2;
  t.X = model->X;
  t.T = model->T;
  t.perm = perm;
  t.loss = loss;
  hipError_t e = launch_mlp_train(t, true, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "mlp_train launch");
  model->adam_t += steps;
  return STOMSFEM_OK;
}

int stomsfem_mlp_grad(const stomsfem_model* model, const float* xb, const float* tb, float* grads, float* loss,
                      void* stream) {
  if (!model || model->kind != 2) return fail(STOMSFEM_EINVAL, "mlp_grad: not a surrogate model");
  if (!device_ptr(xb) || !device_ptr(tb) || !device_ptr(grads))
    return fail(STOMSFEM_EINVAL, "mlp_grad: xb, tb and grads must be device pointers");
  MlpTrainArgs t{};
  t.npatch = model->ncx * model->ncy;
  t.ntrain = MLP_BATCH;
  t.steps = 1;
  t.params = model->params;
  t.xb = xb;
  t.tb = tb;
  t.grads = grads;
  t.loss = loss;
  hipError_t e = launch_mlp_train(t, false, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "mlp_grad launch");
}

int stomsfem_mlp_params(stomsfem_model* model, float* dst, const float* src, void* stream) {
  if (!model || model->kind != 2) return fail(STOMSFEM_EINVAL, "mlp_params: not a surrogate model");
  const size_t bytes = sizeof(float) * (size_t)model->ncx * model->ncy * MLP_NP;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (dst) e = hipMemcpyAsync(dst, model->params, bytes, hipMemcpyDefault, st);
  if (e == hipSuccess && src) e = hipMemcpyAsync(model->params, src, bytes, hipMemcpyDefault, st);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "mlp_params");
}

int stomsfem_mlp_standardization(const stomsfem_model* model, double* mu_host, double* sd_host) {
  if (!model || model->kind != 2) return fail(STOMSFEM_EINVAL, "mlp_standardization: not a surrogate model");
  const size_t bytes = sizeof(double) * model->ncx * model->ncy * 10;
  hipError_t e = hipSuccess;
  if (mu_host) e = hipMemcpy(mu_host, model->mu, bytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess && sd_host) e = hipMemcpy(sd_host, model->sd, bytes, hipMemcpyDeviceToHost);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "mlp_standardization");
}

static int mlp_infer_common(stomsfem_model* model, const double* xi, int32_t nxi, int64_t nsamples, float* Y,
                            double* S, int32_t* status, double tau, int32_t precision, uint64_t* stats,
                            void* stream) {
  if (!model || model->kind != 2) return fail(STOMSFEM_EINVAL, "surrogate: not a surrogate model");
  if (nsamples < 0 || nxi < 1) return fail(STOMSFEM_EINVAL, "surrogate: bad sizes");
  if (model->lv_max >= nxi) return fail(STOMSFEM_EINVAL, "surrogate: nxi smaller than the local variable indices");
  if (precision != STOMSFEM_PREC_F32 && precision != STOMSFEM_PREC_BF16 && precision != STOMSFEM_PREC_F16)
    return fail(STOMSFEM_EINVAL, "surrogate: precision must be STOMSFEM_PREC_F32, _BF16 or _F16");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(xi)) return fail(STOMSFEM_EINVAL, "surrogate: xi must be a device pointer");
  if ((Y && !device_ptr(Y)) || (S && !device_ptr(S)) || (status && !device_ptr(status)) ||
      (stats && !device_ptr(stats)))
    return fail(STOMSFEM_EINVAL, "surrogate: outputs must be device pointers");
  const int Mc = model->ncx * model->ncy;
  OrderedUse order;  // the model's scratch buffers (fallback list, counter, chunk buffers)
  if (int orc = order.begin(model->order_mu, model->order_ev, (hipStream_t)stream); orc != STOMSFEM_OK) return orc;
  if (S) {
    if (model->family == MLP_FAMILY_FEATURES ? nxi < model->nfeat
                                             : (model->fam.g < 1 || model->fam.g * model->fam.g > nxi))
      return fail(STOMSFEM_EINVAL, "surrogate: the model's coefficient family does not match xi");
    const int64_t need = nsamples * Mc;
    if (model->list_cap < need) {
      hipError_t e = hipStreamSynchronize((hipStream_t)stream);
      if (e == hipSuccess) {
        hipFree(model->list);
        model->list = nullptr;
        model->list_cap = 0;
        e = hipMalloc(&model->list, sizeof(int64_t) * need);
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(STOMSFEM_ENOMEM, "surrogate: fallback list allocation failed");
      }
      model->list_cap = need;
    }
  }
  MlpInferArgs a{};
  a.family = model->family;
  a.decades = model->decades;
  a.rw = model->rw;
  a.npatch = Mc;
  a.ncx = model->ncx;
  a.nxi = nxi;
  a.nsamples = nsamples;
  a.params = model->params;
  a.lv = model->lv;
  a.mu = model->mu;
  a.sd = model->sd;
  a.xi = xi;
  a.box = model->box;
  a.tau = tau;
  a.Y = Y;
  a.S = S;
  a.status = status;
  a.count = model->counter;
  a.list = model->list;
  a.stats = (unsigned long long*)stats;
  a.bump_g = model->fam.g;
  a.bump_rho = model->fam.rho;
  a.bump_eps = model->fam.eps;
  a.bump_base = model->fam.base;
  a.bump_amp = model->fam.amp;
  a.bump_beta = model->fam.beta;
  a.m = model->m;
  hipStream_t st = (hipStream_t)stream;
  const int mode = precision == STOMSFEM_PREC_BF16 ? MLP_MODE_BF16
                   : precision == STOMSFEM_PREC_F16  ? MLP_MODE_F16
                                                     : MLP_MODE_F32;
  hipError_t e = launch_mlp_infer(a, mode, st);
  if (e != hipSuccess) return hip_fail(e, "surrogate launch");
  if (!S || (model->m == 8 && model->family == MLP_FAMILY_BUMPS)) return STOMSFEM_OK;
  // plain fallback for m != 8: the listed pairs in chunks (reads the count)
  unsigned long long n = 0;
  e = hipMemcpyAsync(&n, model->counter, sizeof(n), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "surrogate fallback count");
  if (n > (unsigned long long)(nsamples * Mc)) return fail(STOMSFEM_EHIP, "surrogate: fallback count out of range");
  g_surrogate_pairs += (uint64_t)(nsamples * Mc);
  g_surrogate_recomputed += n;
  for (int64_t start = 0; start < (int64_t)n && e == hipSuccess; start += model->chunk) {
    const int64_t cnt = std::min<int64_t>(model->chunk, (int64_t)n - start);
    RegenArgs r{};
    r.ncx = model->ncx;
    r.ncy = model->ncy;
    r.m = model->m;
    r.nxi = nxi;
    r.bp = BumpParams{model->fam.g, model->fam.rho, model->fam.eps, model->fam.base, model->fam.amp, model->fam.beta};
    r.fmap = model->family == MLP_FAMILY_FEATURES ? model->fmap : nullptr;
    r.decades = model->decades;
    r.pairs = model->list + start;
    r.count = cnt;
    r.xi = xi;
    r.out = model->blk;
    e = launch_regen_blocks(r, st);
    if (e == hipSuccess) {
      UpArgs u{};
      u.nsamples = cnt;
      u.ncx = u.ncy = 1;
      u.m = model->m;
      u.npairs = cnt;
      u.a = model->blk;
      u.S = model->Sc;
      u.status = model->stc;
      e = launch_upscale_any(u, STOMSFEM_F64, st);
    }
    if (e == hipSuccess)
      e = launch_mlp_fallback_finish(model->list + start, cnt, model->Sc, model->stc, S, status,
                                     (unsigned long long*)stats, st);
  }
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "surrogate fallback launch");
}

int stomsfem_mlp_gate(const stomsfem_model* model, const float* Y, const double* xi, int32_t nxi, int64_t nsamples,
                      double gate_tol, double* S, int32_t* status, double* gate, void* stream) {
  if (!model || model->kind != 2) return fail(STOMSFEM_EINVAL, "mlp_gate: not a surrogate model");
  if (nsamples < 0 || nxi < 1) return fail(STOMSFEM_EINVAL, "mlp_gate: bad sizes");
  if (model->lv_max >= nxi) return fail(STOMSFEM_EINVAL, "mlp_gate: nxi smaller than the local variable indices");
  if (!(gate_tol >= 0)) return fail(STOMSFEM_EINVAL, "mlp_gate: gate_tol must be >= 0");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(Y) || !device_ptr(xi) || !device_ptr(S))
    return fail(STOMSFEM_EINVAL, "mlp_gate: Y, xi and S must be device pointers");
  if ((status && !device_ptr(status)) || (gate && !device_ptr(gate)))
    return fail(STOMSFEM_EINVAL, "mlp_gate: status and gate must be device pointers");
  MlpInferArgs a{};
  a.family = model->family;
  a.decades = model->decades;
  a.rw = model->rw;
  a.npatch = model->ncx * model->ncy;
  a.ncx = model->ncx;
  a.nxi = nxi;
  a.nsamples = nsamples;
  a.lv = model->lv;
  a.mu = model->mu;
  a.sd = model->sd;
  a.xi = xi;
  a.box = model->box;
  a.tau = gate_tol;
  a.S = S;
  a.status = status;
  a.gate = gate;
  hipError_t e = launch_mlp_gate(a, Y, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "mlp_gate launch");
}

int stomsfem_mlp_predict(const stomsfem_model* model, const double* xi, int32_t nxi, int64_t nsamples, float* Y,
                         int32_t precision, void* stream) {
  if (!Y) return fail(STOMSFEM_EINVAL, "mlp_predict: NULL Y");
  return mlp_infer_common(const_cast<stomsfem_model*>(model), xi, nxi, nsamples, Y, nullptr, nullptr, 0.0, precision,
                          nullptr, stream);
}

int stomsfem_upscale_surrogate(stomsfem_model* model, const double* xi, int32_t nxi, int64_t nsamples, double* S,
                               int32_t* status, double gate_tol, int32_t precision, uint64_t* stats, void* stream) {
  if (!S) return fail(STOMSFEM_EINVAL, "upscale_surrogate: NULL S");
  if (!(gate_tol >= 0)) return fail(STOMSFEM_EINVAL, "upscale_surrogate: gate_tol must be >= 0");
  return mlp_infer_common(model, xi, nxi, nsamples, nullptr, S, status, gate_tol, precision, stats, stream);
}

// ---------------------------------------------------------------------------
// random interpolation
// ---------------------------------------------------------------------------
static BumpParams bump_params(const stomsfem_bump_family& f) {
  return BumpParams{f.g, f.rho, f.eps, f.base, f.amp, f.beta};
}

// Plain solve of `count` listed pairs (p = s * M + K of the model's mesh)
// with coefficients regenerated from xi, in chunks through the model's
// buffers; S[p] and status[p] (code, or the solve's status) are written.
static int ri_plain_pairs(stomsfem_model* md, const int64_t* list, int64_t count, const double* xi, int32_t nxi,
                          double* S, int32_t* status, int32_t code, hipStream_t st) {
  for (int64_t start = 0; start < count; start += md->chunk) {
    const int64_t cnt = std::min(md->chunk, count - start);
    RegenArgs r{};
    r.ncx = md->ncx;
    r.ncy = md->ncy;
    r.m = md->m;
    r.nxi = nxi;
    r.bp = bump_params(md->fam);
    r.pairs = list + start;
    r.count = cnt;
    r.xi = xi;
    r.out = md->blk;
    hipError_t e = launch_regen_blocks(r, st);
    if (e == hipSuccess) {
      UpArgs u{};
      u.nsamples = cnt;
      u.ncx = u.ncy = 1;
      u.m = md->m;
      u.npairs = cnt;
      u.a = md->blk;
      u.S = md->Sc;
      u.status = md->stc;
      e = launch_upscale_any(u, STOMSFEM_F64, st);
    }
    if (e == hipSuccess) e = launch_scatter_pairs(list + start, cnt, md->Sc, md->stc, S, status, code, st);
    if (e != hipSuccess) return hip_fail(e, "interp: plain solve launch");
  }
  return STOMSFEM_OK;
}

int stomsfem_interp_build(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars,
                          const stomsfem_bump_family* fam, int32_t nnodes, double lo, double hi,
                          stomsfem_model** model, void* stream) {
  if (!local_vars || !fam || !model) return fail(STOMSFEM_EINVAL, "interp_build: NULL argument");
  *model = nullptr;
  if (ncx < 1 || ncy < 1 || m < 1 || m > 48) return fail(STOMSFEM_EINVAL, "interp_build: need 1 <= m <= 48");
  if (nnodes < RI_NN_MIN || nnodes > RI_NN_MAX) return fail(STOMSFEM_EINVAL, "interp_build: nnodes must be in 2..9");
  if (!(lo < hi)) return fail(STOMSFEM_EINVAL, "interp_build: need lo < hi");
  if (fam->g < 1 || !(fam->rho > 0) || !(fam->eps > 0)) return fail(STOMSFEM_EINVAL, "interp_build: bad family");
  const int Mc = ncx * ncy, nxi = fam->g * fam->g;
  std::vector<int32_t> nlv(Mc);
  std::vector<int64_t> off(Mc + 1, 0);
  int32_t lv_max = -1;
  for (int K = 0; K < Mc; ++K) {
    int k = 0;
    while (k < RI_KMAX && local_vars[K * RI_KMAX + k] >= 0) ++k;
    for (int i = 0; i < RI_KMAX; ++i) {
      const int32_t j = local_vars[K * RI_KMAX + i];
      if ((i < k && j >= nxi) || (i >= k && j != -1))
        return fail(STOMSFEM_EINVAL, "interp_build: local variables must be < g*g, -1 padded at the end");
      if (i > 0 && i < k && j <= local_vars[K * RI_KMAX + i - 1])
        return fail(STOMSFEM_EINVAL, "interp_build: local variables of a patch must be increasing");
      if (j > lv_max) lv_max = j;
    }
    nlv[K] = k;
    int64_t n = 1;
    for (int i = 0; i < k; ++i) n *= nnodes;
    off[K + 1] = off[K] + n;
  }
  hipStream_t st = (hipStream_t)stream;
  auto* md = new stomsfem_model();
  md->kind = 3;
  hipGetDevice(&md->device);
  md->ncx = ncx;
  md->ncy = ncy;
  md->m = m;
  md->fam = *fam;
  md->lv_max = lv_max;
  md->nn = nnodes;
  md->lo = lo;
  md->hi = hi;
  md->rows = off[Mc];
  md->chunk = std::max<int64_t>(256, std::min<int64_t>(65536, (int64_t{1} << 25) / ((int64_t)m * m)));
  hipError_t e = hipSuccess;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  };
  A((void**)&md->lv, sizeof(int32_t) * Mc * RI_KMAX);
  A((void**)&md->nlv, sizeof(int32_t) * Mc);
  A((void**)&md->off, sizeof(int64_t) * (Mc + 1));
  A((void**)&md->table, sizeof(double) * (size_t)md->rows * 10);
  A((void**)&md->counter, sizeof(unsigned long long));
  A((void**)&md->blk, sizeof(double) * (size_t)md->chunk * m * m);
  A((void**)&md->xin, sizeof(double) * (size_t)md->chunk * nxi);
  A((void**)&md->pairs, sizeof(int64_t) * (size_t)md->chunk);
  A((void**)&md->Sc, sizeof(double) * (size_t)md->chunk * 10);
  A((void**)&md->stc, sizeof(int32_t) * (size_t)md->chunk);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    model_release(md);
    return fail(STOMSFEM_ENOMEM, "interp_build: device allocation failed");
  }
  e = hipMemcpy(md->lv, local_vars, sizeof(int32_t) * Mc * RI_KMAX, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->nlv, nlv.data(), sizeof(int32_t) * Mc, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->off, off.data(), sizeof(int64_t) * (Mc + 1), hipMemcpyHostToDevice);
  std::vector<int32_t> sth;
  int bad = 0;
  for (int64_t start = 0; e == hipSuccess && start < md->rows; start += md->chunk) {
    const int64_t cnt = std::min(md->chunk, md->rows - start);
    RiNodeArgs na{};
    na.npatch = Mc;
    na.nxi = nxi;
    na.nn = nnodes;
    na.lo = lo;
    na.hi = hi;
    na.off = md->off;
    na.lv = md->lv;
    na.nlv = md->nlv;
    na.start = start;
    na.count = cnt;
    na.xi_out = md->xin;
    na.pairs_out = md->pairs;
    e = launch_ri_nodes(na, st);
    if (e != hipSuccess) break;
    RegenArgs r{};
    r.ncx = ncx;
    r.ncy = ncy;
    r.m = m;
    r.nxi = nxi;
    r.bp = bump_params(*fam);
    r.pairs = md->pairs;
    r.count = cnt;
    r.xi = md->xin;
    r.out = md->blk;
    e = launch_regen_blocks(r, st);
    if (e != hipSuccess) break;
    UpArgs u{};
    u.nsamples = cnt;
    u.ncx = u.ncy = 1;
    u.m = m;
    u.npairs = cnt;
    u.a = md->blk;
    u.S = md->table + start * 10;
    u.status = md->stc;
    e = launch_upscale_any(u, STOMSFEM_F64, st);
    if (e != hipSuccess) break;
    sth.resize(cnt);
    e = hipMemcpyAsync(sth.data(), md->stc, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (int64_t i = 0; e == hipSuccess && i < cnt; ++i) bad |= sth[i] != 0;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    model_release(md);
    return hip_fail(e, "interp_build");
  }
  if (bad) {
    model_release(md);
    return fail(STOMSFEM_ENOTSPD, "interp_build: a cell problem at an interpolation node is not positive definite");
  }
  *model = md;
  return STOMSFEM_OK;
}

int stomsfem_interp_apply(stomsfem_model* model, const double* xi, int32_t nxi, int64_t nsamples, double* S,
                          int32_t* status, int64_t* nfallback, void* stream) {
  if (nfallback) *nfallback = 0;
  if (!model || model->kind != 3) return fail(STOMSFEM_EINVAL, "interp_apply: not an interpolation model");
  if (nsamples < 0 || nxi < model->fam.g * model->fam.g)
    return fail(STOMSFEM_EINVAL, "interp_apply: nxi smaller than the family's g*g");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(xi) || !device_ptr(S)) return fail(STOMSFEM_EINVAL, "interp_apply: xi and S must be device pointers");
  if (status && !device_ptr(status)) return fail(STOMSFEM_EINVAL, "interp_apply: status must be a device pointer");
  const int Mc = model->ncx * model->ncy;
  hipStream_t st = (hipStream_t)stream;
  OrderedUse order;  // the model's scratch buffers
  if (int orc = order.begin(model->order_mu, model->order_ev, st); orc != STOMSFEM_OK) return orc;
  const int64_t need = nsamples * Mc;
  if (model->list_cap < need) {
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
      hipFree(model->list);
      model->list = nullptr;
      model->list_cap = 0;
      e = hipMalloc(&model->list, sizeof(int64_t) * need);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(STOMSFEM_ENOMEM, "interp_apply: fallback list allocation failed");
    }
    model->list_cap = need;
  }
  RiApplyArgs a{};
  a.npatch = Mc;
  a.nxi = nxi;
  a.nn = model->nn;
  a.nsamples = nsamples;
  a.lo = model->lo;
  a.hi = model->hi;
  a.table = model->table;
  a.off = model->off;
  a.lv = model->lv;
  a.nlv = model->nlv;
  a.xi = xi;
  a.S = S;
  a.status = status;
  a.list = model->list;
  a.list_count = model->counter;
  hipError_t e = launch_zero_u64(model->counter, st);
  if (e == hipSuccess) e = launch_ri_apply(a, st);
  unsigned long long n = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&n, model->counter, sizeof(n), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "interp_apply");
  if (n > (unsigned long long)need) return fail(STOMSFEM_EHIP, "interp_apply: fallback count out of range");
  if (nfallback) *nfallback = (int64_t)n;
  g_interp_pairs += (uint64_t)need;
  g_interp_fallbacks += n;
  return ri_plain_pairs(model, model->list, (int64_t)n, xi, nxi, S, status, 1, st);
}

// ---------------------------------------------------------------------------
// sparse-grid collocation with search-and-plug-in dictionaries
// ---------------------------------------------------------------------------
// S_K at every table row of a dictionary or interpolation model by the plain
// path: rows of patch K are off[K] .. off[K+1]-1; fill(row, K, x) sets the
// row's local variables in x (the other nxi entries are 0).  Chunks of
// md->chunk pairs; synchronises st per chunk (for the status read).
static int solve_table_rows(stomsfem_model* md, int nxi, const std::vector<int64_t>& off,
                            const std::function<void(int64_t, int, double*)>& fill, hipStream_t st, const char* who) {
  const int Mc = md->ncx * md->ncy;
  std::vector<double> xh;
  std::vector<int64_t> ph;
  std::vector<int32_t> sth;
  int bad = 0, K = 0;
  hipError_t e = hipSuccess;
  for (int64_t start = 0; e == hipSuccess && start < md->rows; start += md->chunk) {
    const int64_t cnt = std::min(md->chunk, md->rows - start);
    xh.assign((size_t)cnt * nxi, 0.0);
    ph.resize(cnt);
    for (int64_t i = 0; i < cnt; ++i) {
      const int64_t row = start + i;
      while (off[K + 1] <= row) ++K;
      fill(row, K, xh.data() + (size_t)i * nxi);
      ph[i] = i * Mc + K;
    }
    e = hipMemcpyAsync(md->xin, xh.data(), sizeof(double) * xh.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(md->pairs, ph.data(), sizeof(int64_t) * cnt, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) break;
    RegenArgs r{};
    r.ncx = md->ncx;
    r.ncy = md->ncy;
    r.m = md->m;
    r.nxi = nxi;
    r.bp = bump_params(md->fam);
    r.pairs = md->pairs;
    r.count = cnt;
    r.xi = md->xin;
    r.out = md->blk;
    e = launch_regen_blocks(r, st);
    if (e != hipSuccess) break;
    UpArgs u{};
    u.nsamples = cnt;
    u.ncx = u.ncy = 1;
    u.m = md->m;
    u.npairs = cnt;
    u.a = md->blk;
    u.S = md->table + start * 10;
    u.status = md->stc;
    e = launch_upscale_any(u, STOMSFEM_F64, st);
    if (e != hipSuccess) break;
    sth.resize(cnt);
    e = hipMemcpyAsync(sth.data(), md->stc, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // also keeps xh, ph alive for the copies
    for (int64_t i = 0; e == hipSuccess && i < cnt; ++i) bad |= sth[i] != 0;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, who);
  if (bad) return fail(STOMSFEM_ENOTSPD, std::string(who) + ": a cell problem at a table node is not positive definite");
  return STOMSFEM_OK;
}

int stomsfem_sparse_grid(int32_t dim, int32_t level, int64_t capacity, int64_t* npoints, int32_t* digits,
                         double* weights) {
  if (!npoints) return fail(STOMSFEM_EINVAL, "sparse_grid: NULL npoints");
  *npoints = 0;
  if (dim < 1 || level < 0 || level > SC_LEVEL_MAX)
    return fail(STOMSFEM_EINVAL, "sparse_grid: need dim >= 1 and 0 <= level <= 8");
  if (sc_term_count(dim, level, 2000000) > 2000000)
    return fail(STOMSFEM_EINVAL, "sparse_grid: more than 2e6 terms in the combination formula");
  std::vector<int32_t> dg;
  std::vector<double> w;
  sc_build_grid(dim, level, dg, w);
  *npoints = (int64_t)w.size();
  if (!digits && !weights) return STOMSFEM_OK;
  if (capacity < *npoints) return fail(STOMSFEM_EINVAL, "sparse_grid: capacity smaller than the number of points");
  if (digits) std::memcpy(digits, dg.data(), sizeof(int32_t) * dg.size());
  if (weights) std::memcpy(weights, w.data(), sizeof(double) * w.size());
  return STOMSFEM_OK;
}

int stomsfem_sc_build(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars,
                      const stomsfem_bump_family* fam, int32_t level, double lo, double hi, const int32_t* digits,
                      int64_t npoints, stomsfem_model** model, void* stream) {
  if (!local_vars || !fam || !model || !digits) return fail(STOMSFEM_EINVAL, "sc_build: NULL argument");
  *model = nullptr;
  if (ncx < 1 || ncy < 1 || m < 1 || m > 48) return fail(STOMSFEM_EINVAL, "sc_build: need 1 <= m <= 48");
  if (level < 0 || level > SC_LEVEL_MAX) return fail(STOMSFEM_EINVAL, "sc_build: need 0 <= level <= 8");
  if (npoints < 1) return fail(STOMSFEM_EINVAL, "sc_build: need at least one collocation point");
  if (!(lo < hi)) return fail(STOMSFEM_EINVAL, "sc_build: need lo < hi");
  if (fam->g < 1 || !(fam->rho > 0) || !(fam->eps > 0)) return fail(STOMSFEM_EINVAL, "sc_build: bad family");
  const int Mc = ncx * ncy, nxi = fam->g * fam->g, D = sc_digit_base(level);
  for (int64_t i = 0; i < npoints * nxi; ++i)
    if (digits[i] < 0 || digits[i] > D) return fail(STOMSFEM_EINVAL, "sc_build: a digit is outside 0..2^max(level,1)");
  std::vector<int32_t> nlv(Mc);
  std::vector<int64_t> off(Mc + 1, 0), keys;
  for (int K = 0; K < Mc; ++K) {
    int k = 0;
    while (k < RI_KMAX && local_vars[K * RI_KMAX + k] >= 0) ++k;
    for (int i = 0; i < RI_KMAX; ++i) {
      const int32_t j = local_vars[K * RI_KMAX + i];
      if ((i < k && j >= nxi) || (i >= k && j != -1))
        return fail(STOMSFEM_EINVAL, "sc_build: local variables must be < g*g, -1 padded at the end");
      if (i > 0 && i < k && j <= local_vars[K * RI_KMAX + i - 1])
        return fail(STOMSFEM_EINVAL, "sc_build: local variables of a patch must be increasing");
    }
    nlv[K] = k;
    // search structure: the distinct local points of K, as sorted keys
    std::vector<int64_t> kk((size_t)npoints);
    for (int64_t p = 0; p < npoints; ++p) {
      int64_t key = 0;
      for (int i = 0; i < k; ++i) key = key * (D + 1) + digits[p * nxi + local_vars[K * RI_KMAX + i]];
      kk[(size_t)p] = key;
    }
    std::sort(kk.begin(), kk.end());
    kk.erase(std::unique(kk.begin(), kk.end()), kk.end());
    keys.insert(keys.end(), kk.begin(), kk.end());
    off[K + 1] = (int64_t)keys.size();
  }
  hipStream_t st = (hipStream_t)stream;
  auto* md = new stomsfem_model();
  md->kind = 4;
  hipGetDevice(&md->device);
  md->ncx = ncx;
  md->ncy = ncy;
  md->m = m;
  md->fam = *fam;
  md->lo = lo;
  md->hi = hi;
  md->sc_level = level;
  md->rows = off[Mc];
  md->chunk = std::max<int64_t>(256, std::min<int64_t>(65536, (int64_t{1} << 25) / ((int64_t)m * m)));
  hipError_t e = hipSuccess;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  };
  A((void**)&md->lv, sizeof(int32_t) * Mc * RI_KMAX);
  A((void**)&md->nlv, sizeof(int32_t) * Mc);
  A((void**)&md->off, sizeof(int64_t) * (Mc + 1));
  A((void**)&md->keys, sizeof(int64_t) * (size_t)md->rows);
  A((void**)&md->table, sizeof(double) * (size_t)md->rows * 10);
  A((void**)&md->blk, sizeof(double) * (size_t)md->chunk * m * m);
  A((void**)&md->xin, sizeof(double) * (size_t)md->chunk * nxi);
  A((void**)&md->pairs, sizeof(int64_t) * (size_t)md->chunk);
  A((void**)&md->stc, sizeof(int32_t) * (size_t)md->chunk);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    model_release(md);
    return fail(STOMSFEM_ENOMEM, "sc_build: device allocation failed");
  }
  e = hipMemcpy(md->lv, local_vars, sizeof(int32_t) * Mc * RI_KMAX, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->nlv, nlv.data(), sizeof(int32_t) * Mc, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->off, off.data(), sizeof(int64_t) * (Mc + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->keys, keys.data(), sizeof(int64_t) * keys.size(), hipMemcpyHostToDevice);
  // offline stage: S_K at every dictionary entry by the plain path, with the
  // local variables at their node values and every other variable 0
  std::vector<double> node(D + 1);
  for (int c = 0; c <= D; ++c) node[c] = lo + (std::cos(M_PI * (double)c / (double)D) + 1.0) * 0.5 * (hi - lo);
  if (e == hipSuccess) {
    const int rc = solve_table_rows(md, nxi, off, [&](int64_t row, int K, double* x) {
      int64_t key = keys[row];
      for (int v = nlv[K] - 1; v >= 0; --v) {
        x[local_vars[K * RI_KMAX + v]] = node[key % (D + 1)];
        key /= (D + 1);
      }
    }, st, "sc_build");
    if (rc != STOMSFEM_OK) {
      model_release(md);
      return rc;
    }
  } else {
    model_release(md);
    return hip_fail(e, "sc_build");
  }
  *model = md;
  return STOMSFEM_OK;
}

int stomsfem_sc_apply(const stomsfem_model* model, const int32_t* digits, int32_t nxi, int64_t npoints, double* S,
                      int32_t* status, void* stream) {
  if (!model || model->kind != 4) return fail(STOMSFEM_EINVAL, "sc_apply: not a collocation model");
  if (npoints < 0 || nxi < model->fam.g * model->fam.g)
    return fail(STOMSFEM_EINVAL, "sc_apply: npoints < 0 or nxi smaller than the family's g*g");
  if (npoints == 0) return STOMSFEM_OK;
  if (!device_ptr(digits) || !device_ptr(S)) return fail(STOMSFEM_EINVAL, "sc_apply: digits and S must be device pointers");
  if (status && !device_ptr(status)) return fail(STOMSFEM_EINVAL, "sc_apply: status must be a device pointer");
  ScApplyArgs a{};
  a.npatch = model->ncx * model->ncy;
  a.nxi = nxi;
  a.D = sc_digit_base(model->sc_level);
  a.npoints = npoints;
  a.digits = digits;
  a.lv = model->lv;
  a.nlv = model->nlv;
  a.off = model->off;
  a.keys = model->keys;
  a.table = model->table;
  a.S = S;
  a.status = status;
  hipError_t e = launch_sc_apply(a, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "sc_apply launch");
}

int stomsfem_quadrature(const double* U, const double* w, int64_t npoints, int32_t nu, double* mean, double* var,
                        void* stream) {
  if (npoints < 1 || nu < 1) return fail(STOMSFEM_EINVAL, "quadrature: need npoints >= 1 and nu >= 1");
  if (!device_ptr(U) || !device_ptr(w)) return fail(STOMSFEM_EINVAL, "quadrature: U and w must be device pointers");
  if ((mean && !device_ptr(mean)) || (var && !device_ptr(var)))
    return fail(STOMSFEM_EINVAL, "quadrature: mean and var must be device pointers");
  void* work = nullptr;
  WorkspaceLease lease;
  int rc = lease.acquire(sizeof(double) * (size_t)sc_quad_work_doubles(npoints, nu), (hipStream_t)stream, &work);
  if (rc != STOMSFEM_OK) return rc;
  hipError_t e = launch_sc_quadrature(U, w, npoints, nu, mean, var, (double*)work, (hipStream_t)stream);
  return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "quadrature launch");
}

int stomsfem_sgi_build(int32_t ncx, int32_t ncy, int32_t m, const int32_t* local_vars,
                       const stomsfem_bump_family* fam, int32_t level, double lo, double hi, stomsfem_model** model,
                       void* stream) {
  if (!local_vars || !fam || !model) return fail(STOMSFEM_EINVAL, "sgi_build: NULL argument");
  *model = nullptr;
  if (ncx < 1 || ncy < 1 || m < 1 || m > 48) return fail(STOMSFEM_EINVAL, "sgi_build: need 1 <= m <= 48");
  if (level < 0 || level > SGI_LEVEL_MAX) return fail(STOMSFEM_EINVAL, "sgi_build: need 0 <= level <= 5");
  if (!(lo < hi)) return fail(STOMSFEM_EINVAL, "sgi_build: need lo < hi");
  if (fam->g < 1 || !(fam->rho > 0) || !(fam->eps > 0)) return fail(STOMSFEM_EINVAL, "sgi_build: bad family");
  const int Mc = ncx * ncy, nxi = fam->g * fam->g, D = sc_digit_base(level);
  std::vector<int32_t> nlv(Mc);
  int kmax = 1;
  for (int K = 0; K < Mc; ++K) {
    int k = 0;
    while (k < RI_KMAX && local_vars[K * RI_KMAX + k] >= 0) ++k;
    for (int i = 0; i < RI_KMAX; ++i) {
      const int32_t j = local_vars[K * RI_KMAX + i];
      if ((i < k && j >= nxi) || (i >= k && j != -1))
        return fail(STOMSFEM_EINVAL, "sgi_build: local variables must be < g*g, -1 padded at the end");
      if (i > 0 && i < k && j <= local_vars[K * RI_KMAX + i - 1])
        return fail(STOMSFEM_EINVAL, "sgi_build: local variables of a patch must be increasing");
    }
    nlv[K] = k;
    kmax = std::max(kmax, k);
  }
  SgiComb C;
  sgi_combination(level, C);
  const auto& gdig = C.gdig;
  const auto& npts = C.npts;
  const auto& lofs = C.lofs;
  const auto& nodes = C.nodes;
  const auto& cc = C.cc;
  const auto& cbo = C.cbo;
  const auto& rows_all = C.rows_all;
  const auto& rofs = C.rofs;
  const bool missing = C.missing;
  const int nb = (int)nodes.size();
  if (missing) return fail(STOMSFEM_EINVAL, "sgi_build: a tensor node of the combination is not a grid node");
  std::vector<int64_t> off(Mc + 1, 0);
  for (int K = 0; K < Mc; ++K) off[K + 1] = off[K] + npts[nlv[K]];
  hipStream_t st = (hipStream_t)stream;
  auto* md = new stomsfem_model();
  md->kind = 5;
  hipGetDevice(&md->device);
  md->ncx = ncx;
  md->ncy = ncy;
  md->m = m;
  md->fam = *fam;
  md->lo = lo;
  md->hi = hi;
  md->sc_level = level;
  md->rows = off[Mc];
  md->sg_nb = nb;
  md->sg_kmax = kmax;
  std::memcpy(md->sg_lofs, lofs, sizeof(lofs));
  std::memcpy(md->sg_rofs, rofs, sizeof(rofs));
  md->chunk = std::max<int64_t>(256, std::min<int64_t>(65536, (int64_t{1} << 25) / ((int64_t)m * m)));
  hipError_t e = hipSuccess;
  auto A = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes);
  };
  A((void**)&md->lv, sizeof(int32_t) * Mc * RI_KMAX);
  A((void**)&md->nlv, sizeof(int32_t) * Mc);
  A((void**)&md->off, sizeof(int64_t) * (Mc + 1));
  A((void**)&md->table, sizeof(double) * (size_t)md->rows * 10);
  A((void**)&md->counter, sizeof(unsigned long long));
  A((void**)&md->blk, sizeof(double) * (size_t)md->chunk * m * m);
  A((void**)&md->xin, sizeof(double) * (size_t)md->chunk * nxi);
  A((void**)&md->pairs, sizeof(int64_t) * (size_t)md->chunk);
  A((void**)&md->Sc, sizeof(double) * (size_t)md->chunk * 10);
  A((void**)&md->stc, sizeof(int32_t) * (size_t)md->chunk);
  A((void**)&md->cb_coef, sizeof(double) * cc.size());
  A((void**)&md->cb_boff, sizeof(uint32_t) * cbo.size());
  A((void**)&md->cb_rows, sizeof(int32_t) * rows_all.size());
  A((void**)&md->sg_nodes, sizeof(double) * nodes.size());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    model_release(md);
    return fail(STOMSFEM_ENOMEM, "sgi_build: device allocation failed");
  }
  e = hipMemcpy(md->lv, local_vars, sizeof(int32_t) * Mc * RI_KMAX, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->nlv, nlv.data(), sizeof(int32_t) * Mc, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->off, off.data(), sizeof(int64_t) * (Mc + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->cb_coef, cc.data(), sizeof(double) * cc.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->cb_boff, cbo.data(), sizeof(uint32_t) * cbo.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(md->cb_rows, rows_all.data(), sizeof(int32_t) * rows_all.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(md->sg_nodes, nodes.data(), sizeof(double) * nodes.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    model_release(md);
    return hip_fail(e, "sgi_build");
  }
  const int rc = solve_table_rows(md, nxi, off, [&](int64_t row, int K, double* x) {
    const int k = nlv[K];
    const int64_t r = row - off[K];
    for (int v = 0; v < k; ++v) {
      const int32_t c = gdig[k][r * k + v];
      x[local_vars[K * RI_KMAX + v]] = lo + (std::cos(M_PI * (double)c / (double)D) + 1.0) * 0.5 * (hi - lo);
    }
  }, st, "sgi_build");
  if (rc != STOMSFEM_OK) {
    model_release(md);
    return rc;
  }
  *model = md;
  return STOMSFEM_OK;
}

int stomsfem_sgi_apply(stomsfem_model* model, const double* xi, int32_t nxi, int64_t nsamples, double* S,
                       int32_t* status, int64_t* nfallback, void* stream) {
  if (nfallback) *nfallback = 0;
  if (!model || model->kind != 5) return fail(STOMSFEM_EINVAL, "sgi_apply: not a sparse-grid interpolation model");
  if (nsamples < 0 || nxi < model->fam.g * model->fam.g)
    return fail(STOMSFEM_EINVAL, "sgi_apply: nsamples < 0 or nxi smaller than the family's g*g");
  if (nsamples == 0) return STOMSFEM_OK;
  if (!device_ptr(xi) || !device_ptr(S)) return fail(STOMSFEM_EINVAL, "sgi_apply: xi and S must be device pointers");
  if (status && !device_ptr(status)) return fail(STOMSFEM_EINVAL, "sgi_apply: status must be a device pointer");
  const int Mc = model->ncx * model->ncy;
  if (Mc > 65535) return fail(STOMSFEM_EINVAL, "sgi_apply: at most 65535 coarse elements");
  hipStream_t st = (hipStream_t)stream;
  OrderedUse order;  // the model's scratch buffers
  if (int orc = order.begin(model->order_mu, model->order_ev, st); orc != STOMSFEM_OK) return orc;
  const int64_t need = nsamples * Mc;
  if (model->list_cap < need) {
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
      hipFree(model->list);
      model->list = nullptr;
      model->list_cap = 0;
      e = hipMalloc(&model->list, sizeof(int64_t) * need);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(STOMSFEM_ENOMEM, "sgi_apply: fallback list allocation failed");
    }
    model->list_cap = need;
  }
  SgiApplyArgs a{};
  a.npatch = Mc;
  a.nxi = nxi;
  a.level = model->sc_level;
  a.nb = model->sg_nb;
  a.kmax = model->sg_kmax;
  a.nsamples = nsamples;
  a.lo = model->lo;
  a.hi = model->hi;
  a.table = model->table;
  a.off = model->off;
  a.lv = model->lv;
  a.nlv = model->nlv;
  a.nodes = model->sg_nodes;
  std::memcpy(a.lofs, model->sg_lofs, sizeof(a.lofs));
  std::memcpy(a.rofs, model->sg_rofs, sizeof(a.rofs));
  a.cb_coef = model->cb_coef;
  a.cb_boff = model->cb_boff;
  a.cb_rows = model->cb_rows;
  a.xi = xi;
  a.S = S;
  a.status = status;
  a.list = model->list;
  a.list_count = model->counter;
  hipError_t e = launch_zero_u64(model->counter, st);
  if (e == hipSuccess) e = launch_sgi_apply(a, st);
  unsigned long long n = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&n, model->counter, sizeof(n), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "sgi_apply");
  if (n > (unsigned long long)need) return fail(STOMSFEM_EHIP, "sgi_apply: fallback count out of range");
  if (nfallback) *nfallback = (int64_t)n;
  return ri_plain_pairs(model, model->list, (int64_t)n, xi, nxi, S, status, 1, st);
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
static int time_launches(const std::function<int()>& launch, int reps, hipStream_t st, double* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int rc = e == hipSuccess ? launch() : STOMSFEM_EHIP;  // warm-up
  if (rc == STOMSFEM_OK && e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && rc == STOMSFEM_OK && e == hipSuccess; ++r) rc = launch();
  if (rc == STOMSFEM_OK && e == hipSuccess) e = hipEventRecord(e1, st);
  if (rc == STOMSFEM_OK && e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.0f;
  if (rc == STOMSFEM_OK && e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (rc != STOMSFEM_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "autotune timing");
  *ms = (double)t / reps;
  return STOMSFEM_OK;
}

int stomsfem_autotune(const stomsfem_batch* batch, int32_t reps, stomsfem_tuning* out, void* stream) {
  if (!batch || reps < 1) return fail(STOMSFEM_EINVAL, "autotune: NULL batch or reps < 1");
  int rc = check_batch(*batch, 0);
  if (rc != STOMSFEM_OK) return rc;
  if (batch->nsamples == 0) return fail(STOMSFEM_EINVAL, "autotune: empty batch");
  hipStream_t st = (hipStream_t)stream;
  const stomsfem_batch& b = *batch;
  const UpArgs up = to_args(b);
  const int64_t M = (int64_t)b.ncx * b.ncy;
  const size_t sbytes = sizeof(double) * 10 * (size_t)up.npairs;
  // 1. launch shape on the whole batch; every variant must reproduce the
  //    default variant bit for bit (same arithmetic per pair)
  std::vector<LaunchCfg> shapes;
  if (b.m <= 8) {
    for (int bs : {64, 128, 256}) shapes.push_back(LaunchCfg{bs, 1});
  } else if (tiled_supports(b.m)) {
    for (int wv : {1, 2}) shapes.push_back(LaunchCfg{64, wv});
  } else {
    shapes.push_back(LaunchCfg{});
  }
  std::vector<unsigned char> ref(sbytes), got(sbytes);
  double best_ms = 0.0, default_ms = 0.0;
  LaunchCfg best = shapes[0];
  for (size_t i = 0; i < shapes.size(); ++i) {
    double ms = 0.0;
    const LaunchCfg c = shapes[i];
    rc = time_launches([&]() {
      hipError_t e = launch_upscale_cfg(up, b.a_dtype, st, c);
      return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "autotune launch");
    }, reps, st, &ms);
    if (rc != STOMSFEM_OK) return rc;
    hipError_t e = hipMemcpy(i == 0 ? ref.data() : got.data(), b.S, sbytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "autotune copy");
    if (i > 0 && got != ref) continue;  // a shape that changes the result is never chosen
    if (i == 0) default_ms = ms;
    if (i == 0 || ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  // 2. precision variant on a prefix of the samples (the refined variant can
  //    be much slower); it must agree with FP64 to the refinement tolerance
  best.precision = STOMSFEM_PREC_F64;
  if (b.m <= 32) {
    int dev = 0, maxlds = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (upscale_mixed_lds_bytes(b.m) + 256 <= (size_t)maxlds) {
      stomsfem_batch sub = b;
      sub.nsamples = std::max<int64_t>(1, std::min<int64_t>(b.nsamples, (16384 + M - 1) / M));
      const size_t sub_bytes = sizeof(double) * 10 * (size_t)(sub.nsamples * M);
      double ms64 = 0.0, ms32 = 0.0;
      rc = time_launches([&]() {
        hipError_t e = launch_upscale_cfg(to_args(sub), sub.a_dtype, st, best);
        return e == hipSuccess ? STOMSFEM_OK : hip_fail(e, "autotune launch");
      }, reps, st, &ms64);
      if (rc != STOMSFEM_OK) return rc;
      std::vector<double> s64(sub_bytes / 8), s32(sub_bytes / 8);
      hipError_t e = hipMemcpy(s64.data(), b.S, sub_bytes, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(e, "autotune copy");
      rc = time_launches([&]() { return upscale_refined(sub, st); }, reps, st, &ms32);
      if (rc != STOMSFEM_OK) return rc;
      e = hipMemcpy(s32.data(), b.S, sub_bytes, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(e, "autotune copy");
      bool agree = true;
      for (size_t p = 0; p < s64.size() / 10 && agree; ++p) {
        double d = 0.0, sc = 0.0;
        for (int q = 0; q < 10; ++q) {
          d = std::max(d, std::fabs(s64[p * 10 + q] - s32[p * 10 + q]));
          sc = std::max(sc, std::fabs(s64[p * 10 + q]));
        }
        agree = d <= 1e-10 * sc;
      }
      if (agree && ms32 < ms64) best.precision = STOMSFEM_PREC_F32_REFINE64;
    }
  }
  // leave the batch's S from the chosen configuration
  if (best.precision == STOMSFEM_PREC_F32_REFINE64) {
    rc = upscale_refined(b, st);
    if (rc != STOMSFEM_OK) return rc;
  } else {
    hipError_t e = launch_upscale_cfg(up, b.a_dtype, st, best);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "autotune final launch");
  }
  best.ms_default = default_ms;
  best.ms_best = best_ms;
  best.tuned = 1;
  {
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_tune_mx);
    g_tune[{dev, b.m, b.a_dtype}] = best;
  }
  if (out) {
    out->m = b.m;
    out->a_dtype = b.a_dtype;
    out->lane_block = best.lane_block;
    out->tiled_waves = best.tiled_waves;
    out->precision = best.precision;
    out->ms_default = default_ms;
    out->ms_best = best_ms;
    out->candidates = (int32_t)shapes.size();
  }
  return STOMSFEM_OK;
}

int stomsfem_tuning_reset(void) {
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tune_mx);
  for (auto it = g_tune.begin(); it != g_tune.end();) {
    if (std::get<0>(it->first) == dev) it = g_tune.erase(it);
    else ++it;
  }
  return STOMSFEM_OK;
}

// ---------------------------------------------------------------------------
// counters, training alias, model files
// ---------------------------------------------------------------------------
int stomsfem_stats_get(stomsfem_stats* out) {
  if (!out) return fail(STOMSFEM_EINVAL, "stats_get: NULL");
  out->refine_pairs = g_refine_pairs.load();
  out->refine_recomputed = g_refine_recomputed.load();
  out->interp_pairs = g_interp_pairs.load();
  out->interp_fallbacks = g_interp_fallbacks.load();
  out->surrogate_pairs = g_surrogate_pairs.load();
  out->surrogate_recomputed = g_surrogate_recomputed.load();
  return STOMSFEM_OK;
}

int stomsfem_stats_reset(void) {
  g_refine_pairs = 0;
  g_refine_recomputed = 0;
  g_interp_pairs = 0;
  g_interp_fallbacks = 0;
  g_surrogate_pairs = 0;
  g_surrogate_recomputed = 0;
  return STOMSFEM_OK;
}

int stomsfem_model_shape(const stomsfem_model* model, int32_t* kind, int32_t* ncx, int32_t* ncy, int32_t* m) {
  if (!model) return fail(STOMSFEM_EINVAL, "model_shape: NULL model");
  if (kind) *kind = model->kind;
  if (ncx) *ncx = model->ncx;
  if (ncy) *ncy = model->ncy;
  if (m) *m = model->kind == 9 ? model->os_m : model->m;
  return STOMSFEM_OK;
}

int stomsfem_surrogate_train(stomsfem_model* model, int32_t steps, float lr, const int64_t* perm, float* loss,
                             void* stream) {
  return stomsfem_mlp_train(model, steps, lr, perm, loss, stream);
}

namespace {
struct ModelFileHeader {
  char magic[8];
  uint32_t abi, kind;
  int32_t ncx, ncy, m, nn;
  int32_t rmax, KD, PP, lv_max;
  int64_t rows, adam_t;
  double box, lo, hi;
  stomsfem_bump_family fam;
};
struct ArrayRecord {
  uint32_t id, elem;
  uint64_t count;
};
const char kModelMagic[8] = {'S', 'T', 'O', 'M', 'S', 'F', 'E', 'M'};

struct ArraySpec {
  void** dev;
  size_t elem;
  size_t count;
};

std::vector<ArraySpec> model_arrays(stomsfem_model* md) {
  const size_t M = (size_t)md->ncx * md->ncy, nI = (size_t)(md->m - 1) * (md->m - 1);
  switch (md->kind) {
    case 1:
      return {{(void**)&md->rK, 4, M},
              {(void**)&md->lambda, 8, M * nI},
              {(void**)&md->Z, 8, M * nI * md->rmax},
              {(void**)&md->phibar, 8, M * 3 * nI},
              {(void**)&md->G32, 4, M * md->KD * md->PP},
              {(void**)&md->G64, 8, M * md->KD * md->PP}};
    case 2:
      return {{(void**)&md->lv, 4, M * MLP_KIN},   {(void**)&md->params, 4, M * MLP_NP},
              {(void**)&md->m1, 4, M * MLP_NP},    {(void**)&md->m2, 4, M * MLP_NP},
              {(void**)&md->mu, 8, M * 10},        {(void**)&md->sd, 8, M * 10},
              {(void**)&md->sd_raw, 8, M * 10}};
    case 3:
      return {{(void**)&md->lv, 4, M * RI_KMAX},
              {(void**)&md->nlv, 4, M},
              {(void**)&md->off, 8, M + 1},
              {(void**)&md->table, 8, (size_t)md->rows * 10}};
    case 9:
      return {{(void**)&md->rK, 4, M},
              {(void**)&md->lambda, 8, M * nI},
              {(void**)&md->Z, 8, M * nI * md->rmax},
              {(void**)&md->phibar, 8, M * 3 * nI},
              {(void**)&md->GO32, 4, M * md->KD * RBO_PO},
              {(void**)&md->GO, 8, M * md->KD * RBO_PO},
              {(void**)&md->Pc, 8, M * 4 * RBO_NF}};
    default:
      return {};
  }
}
}  // namespace

int stomsfem_model_save(const stomsfem_model* model, const char* path) {
  if (!model || !path) return fail(STOMSFEM_EINVAL, "model_save: NULL argument");
  if ((model->kind < 1 || model->kind > 3) && model->kind != 9)
    return fail(STOMSFEM_EINVAL, "model_save: unknown model kind");
  if (model->family != MLP_FAMILY_BUMPS)
    return fail(STOMSFEM_EINVAL, "model_save: surrogates of the channels medium are not saved");
  ModelFileHeader h{};
  std::memcpy(h.magic, kModelMagic, 8);
  h.abi = STOMSFEM_ABI_VERSION;
  h.kind = (uint32_t)model->kind;
  h.ncx = model->ncx;
  h.ncy = model->ncy;
  h.m = model->m;
  h.nn = model->nn;
  h.rmax = model->rmax;
  h.KD = model->KD;
  h.PP = model->PP;
  h.lv_max = model->lv_max;
  if (model->kind == 9) {  // the oversampling and the element side travel in nn and lv_max
    h.nn = model->os_o;
    h.lv_max = model->os_m;
  }
  h.rows = model->rows;
  h.adam_t = model->adam_t;
  h.box = model->box;
  h.lo = model->lo;
  h.hi = model->hi;
  h.fam = model->fam;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "model_save");
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(STOMSFEM_EINVAL, std::string("model_save: cannot open ") + path);
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
  uint32_t id = 0;
  for (const ArraySpec& a : model_arrays(const_cast<stomsfem_model*>(model))) {
    std::vector<unsigned char> buf(a.elem * a.count);
    if (ok && !buf.empty()) ok = hipMemcpy(buf.data(), *a.dev, buf.size(), hipMemcpyDeviceToHost) == hipSuccess;
    const ArrayRecord r{id++, (uint32_t)a.elem, (uint64_t)a.count};
    ok = ok && std::fwrite(&r, sizeof(r), 1, f) == 1;
    if (ok && !buf.empty()) ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
  }
  ok = (std::fclose(f) == 0) && ok;
  return ok ? STOMSFEM_OK : fail(STOMSFEM_EHIP, std::string("model_save: write to ") + path + " failed");
}

int stomsfem_model_load(const char* path, stomsfem_model** model) {
  if (!path || !model) return fail(STOMSFEM_EINVAL, "model_load: NULL argument");
  *model = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(STOMSFEM_EINVAL, std::string("model_load: cannot open ") + path);
  ModelFileHeader h{};
  if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, kModelMagic, 8) != 0) {
    std::fclose(f);
    return fail(STOMSFEM_EVERSION, "model_load: not a model file");
  }
  if (h.abi != STOMSFEM_ABI_VERSION) {
    std::fclose(f);
    return fail(STOMSFEM_EVERSION, "model_load: written by ABI version " + std::to_string(h.abi));
  }
  const bool sane = ((h.kind >= 1 && h.kind <= 3) || h.kind == 9) && h.ncx >= 1 && h.ncy >= 1 && h.ncx <= 4096 &&
                    h.ncy <= 4096 && h.m >= 1 && (h.m <= 48 || (h.kind == 9 && h.m <= 64)) && h.rows >= 0 && h.rmax >= 0 && h.rmax <= 8 &&
                    h.KD >= 0 && h.PP >= 0 && h.KD <= 4096 && h.PP <= 4096 &&
                    (h.kind != 3 || (h.nn >= RI_NN_MIN && h.nn <= RI_NN_MAX)) &&
                    (h.kind != 9 || (h.m >= 2 && h.m <= 64 && h.rmax == 8 && h.nn >= 0 && h.lv_max >= 1 &&
                                     h.lv_max + 2 * h.nn == h.m && h.KD == rb_pad_kd(h.m)));
  if (!sane) {
    std::fclose(f);
    return fail(STOMSFEM_EINVAL, "model_load: corrupt header");
  }
  auto* md = new stomsfem_model();
  hipGetDevice(&md->device);
  md->kind = (int)h.kind;
  md->ncx = h.ncx;
  md->ncy = h.ncy;
  md->m = h.m;
  md->nn = h.nn;
  md->rmax = h.rmax;
  md->KD = h.KD;
  md->PP = h.PP;
  md->lv_max = h.lv_max;
  md->rows = h.rows;
  md->adam_t = h.adam_t;
  md->box = h.box;
  md->lo = h.lo;
  md->hi = h.hi;
  md->fam = h.fam;
  if (md->kind == 9) {
    md->os_o = h.nn;
    md->os_m = h.lv_max;
    md->nn = 0;
    md->lv_max = -1;
  }
  int rc = STOMSFEM_OK;
  uint32_t id = 0;
  for (const ArraySpec& a : model_arrays(md)) {
    ArrayRecord r{};
    if (std::fread(&r, sizeof(r), 1, f) != 1 || r.id != id++ || r.elem != a.elem || r.count != a.count) {
      rc = fail(STOMSFEM_EINVAL, "model_load: array table does not match the header");
      break;
    }
    std::vector<unsigned char> buf(a.elem * a.count);
    if (!buf.empty() && std::fread(buf.data(), 1, buf.size(), f) != buf.size()) {
      rc = fail(STOMSFEM_EINVAL, "model_load: truncated file");
      break;
    }
    if (hipMalloc(a.dev, std::max<size_t>(buf.size(), 8)) != hipSuccess) {
      (void)hipGetLastError();
      *a.dev = nullptr;
      rc = fail(STOMSFEM_ENOMEM, "model_load: device allocation failed");
      break;
    }
    if (!buf.empty() && hipMemcpy(*a.dev, buf.data(), buf.size(), hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(STOMSFEM_EHIP, "model_load: copy failed");
      break;
    }
  }
  std::fclose(f);
  // work buffers of the online stages, as the constructors make them
  if (rc == STOMSFEM_OK && (md->kind == 2 || md->kind == 3)) {
    hipError_t e = hipMalloc((void**)&md->counter, sizeof(unsigned long long));
    const int m = md->m;
    const bool chunked = md->kind == 3 || m != 8;
    if (chunked) {
      md->chunk = std::max<int64_t>(256, std::min<int64_t>(65536, (int64_t{1} << 25) / ((int64_t)m * m)));
      if (e == hipSuccess) e = hipMalloc((void**)&md->blk, sizeof(double) * (size_t)md->chunk * m * m);
      if (e == hipSuccess) e = hipMalloc((void**)&md->Sc, sizeof(double) * (size_t)md->chunk * 10);
      if (e == hipSuccess) e = hipMalloc((void**)&md->stc, sizeof(int32_t) * (size_t)md->chunk);
    }
    if (md->kind == 3) {
      const int nxi = std::max(1, md->fam.g * md->fam.g);
      if (e == hipSuccess) e = hipMalloc((void**)&md->xin, sizeof(double) * (size_t)md->chunk * nxi);
      if (e == hipSuccess) e = hipMalloc((void**)&md->pairs, sizeof(int64_t) * (size_t)md->chunk);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      rc = fail(STOMSFEM_ENOMEM, "model_load: device allocation failed");
    }
  }
  if (rc != STOMSFEM_OK) {
    model_release(md);
    return rc;
  }
  *model = md;
  return STOMSFEM_OK;
}

int stomsfem_workspace_reserve(int64_t bytes) {
  if (bytes < 0) return fail(STOMSFEM_EINVAL, "workspace_reserve: bytes < 0");
  if (bytes == 0) return STOMSFEM_OK;
  int rc = STOMSFEM_OK;
  Workspace* w = workspace_of_current_device(&rc);
  if (!w) return rc;
  std::lock_guard<std::mutex> lk(w->lease);
  return workspace_grow(*w, (size_t)bytes);
}

int stomsfem_workspace_release(void) {
  int rc = STOMSFEM_OK;
  Workspace* w = workspace_of_current_device(&rc);
  if (!w) return rc;
  std::lock_guard<std::mutex> lk(w->lease);
  if (w->ptr) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    hipFree(w->ptr);
    w->ptr = nullptr;
    w->bytes = 0;
  }
  return STOMSFEM_OK;
}

}  // extern "C"
