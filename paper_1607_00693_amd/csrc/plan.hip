// Execution plans: a list of stages (one sample batch each: coefficient
// generation, local upscaling, coarse solve and quantity of interest, i.e.
// Sec. 2.2 eqs. MsFEB, stiffness_local, upscaleSUF and the Monte Carlo mean
// of Sec. 4.1.1) captured once into HIP graphs and replayed.
//
// Stages are grouped by H/h: each group owns its device buffers (coefficient
// field, S, per-pair status, coarse workspace) sized for its largest stage,
// and its stages run in order on the group's stream.  The whole-plan graph
// forks one branch per group from a common start and joins them, so batches
// of different H/h run concurrently (each kernel keeps its own resource
// footprint; the hardware packs workgroups of several kernels onto the CUs).
// A per-stage graph of every stage serves latency measurements.  Nothing is
// allocated, freed or synchronised while a plan is replayed.
#include <string>
#include <vector>

#include "common.h"

namespace stomsfem {
hipError_t launch_upscale_any(const UpArgs& args, int a_dtype, hipStream_t st);
hipError_t launch_coarse(int ncx, int ncy, int64_t N, const double* S, const double* load, double* U, double* mean,
                         double* var, int32_t* status, double* work, hipStream_t st);
int64_t coarse_work_doubles(int ncx, int ncy, int64_t nsamples);
size_t coarse_lds_bytes(int ncx, bool pg);
hipError_t launch_coef_bumps(int64_t nsamples, int nfine, const double* xi, int nxi, int g, double rho, double eps,
                             double base, double amp, double beta, void* a, int a_dtype, hipStream_t st);
hipError_t launch_coef_features(int64_t nsamples, int nfine, const int32_t* map, int nfeat, const double* xi, int nxi,
                                double decades, void* a, int a_dtype, hipStream_t st);
void set_last_error(const std::string& msg);
}  // namespace stomsfem

using namespace stomsfem;

struct stomsfem_plan {
  struct Group {
    int m = 0, ncx = 0, ncy = 0;
    void* a = nullptr;
    double* S = nullptr;
    int32_t* status = nullptr;
    int32_t* cstatus = nullptr;
    double* work = nullptr;
    double* U = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<int> stages;
  };
  int device = 0;
  std::vector<stomsfem_stage> stages;
  std::vector<int> group_of;
  std::vector<Group> groups;
  hipStream_t capture = nullptr;
  hipEvent_t fork = nullptr;
  hipGraph_t g_all = nullptr;
  hipGraphExec_t x_all = nullptr;
  std::vector<hipGraph_t> g_stage;
  std::vector<hipGraphExec_t> x_stage;
};

namespace {

void plan_release(stomsfem_plan* p) {
  if (!p) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(p->device);
  hipDeviceSynchronize();
  for (auto x : p->x_stage)
    if (x) hipGraphExecDestroy(x);
  for (auto g : p->g_stage)
    if (g) hipGraphDestroy(g);
  if (p->x_all) hipGraphExecDestroy(p->x_all);
  if (p->g_all) hipGraphDestroy(p->g_all);
  for (auto& g : p->groups) {
    hipFree(g.a);
    hipFree(g.S);
    hipFree(g.status);
    hipFree(g.cstatus);
    hipFree(g.work);
    hipFree(g.U);
    if (g.stream) hipStreamDestroy(g.stream);
    if (g.done) hipEventDestroy(g.done);
  }
  if (p->fork) hipEventDestroy(p->fork);
  if (p->capture) hipStreamDestroy(p->capture);
  hipSetDevice(cur);
  delete p;
}

// Enqueue stage i of the plan on stream st (no allocation, no synchronisation).
hipError_t enqueue_stage(const stomsfem_plan* p, int i, hipStream_t st) {
  const stomsfem_stage& s = p->stages[i];
  const stomsfem_plan::Group& g = p->groups[p->group_of[i]];
  const int nfine = s.ncx * s.m;
  hipError_t e;
  if (s.family == STOMSFEM_FAMILY_BUMPS)
    e = launch_coef_bumps(s.nsamples, nfine, s.xi, s.nxi, s.bumps.g, s.bumps.rho, s.bumps.eps, s.bumps.base,
                          s.bumps.amp, s.bumps.beta, g.a, s.a_dtype, st);
  else
    e = launch_coef_features(s.nsamples, nfine, s.feature_map, s.nfeat, s.xi, s.nxi, s.decades, g.a, s.a_dtype, st);
  if (e != hipSuccess) return e;
  UpArgs up{};
  up.nsamples = s.nsamples;
  up.ncx = s.ncx;
  up.ncy = s.ncy;
  up.m = s.m;
  up.npairs = s.nsamples * (int64_t)s.ncx * s.ncy;
  up.a = g.a;
  up.S = g.S;
  up.status = s.status ? s.status : g.status;
  e = launch_upscale_any(up, s.a_dtype, st);
  if (e != hipSuccess) return e;
  return launch_coarse(s.ncx, s.ncy, s.nsamples, g.S, nullptr, s.U ? s.U : g.U, s.qoi_mean, s.qoi_var, g.cstatus,
                       g.work, st);
}

int pfail(int code, const std::string& msg) {
  set_last_error(msg);
  return code;
}

}  // namespace

extern "C" {

int stomsfem_plan_create(const stomsfem_stage* stages, int32_t nstage, stomsfem_plan** plan) {
  if (!plan || nstage < 1 || !stages) return pfail(STOMSFEM_EINVAL, "plan_create: need at least one stage");
  *plan = nullptr;
  for (int i = 0; i < nstage; ++i) {
    const stomsfem_stage& s = stages[i];
    const std::string w = "plan_create: stage " + std::to_string(i) + ": ";
    if (s.ncx < 2 || s.ncx != s.ncy) return pfail(STOMSFEM_EINVAL, w + "need a square coarse mesh with ncx >= 2");
    if (s.m < 1 || s.m > 48) return pfail(STOMSFEM_EINVAL, w + "m must be in 1..48");
    if (s.nsamples < 1) return pfail(STOMSFEM_EINVAL, w + "nsamples must be >= 1");
    if (s.a_dtype != STOMSFEM_F64 && s.a_dtype != STOMSFEM_F32) return pfail(STOMSFEM_EINVAL, w + "bad a_dtype");
    if (coarse_lds_bytes(s.ncx, false) > 64 * 1024) return pfail(STOMSFEM_EINVAL, w + "coarse mesh too large");
    if (!s.xi) return pfail(STOMSFEM_EINVAL, w + "xi is NULL");
    if (s.family == STOMSFEM_FAMILY_BUMPS) {
      if (s.bumps.g < 1 || s.nxi < s.bumps.g * s.bumps.g || !(s.bumps.rho > 0) || !(s.bumps.eps > 0))
        return pfail(STOMSFEM_EINVAL, w + "bad bump family");
    } else if (s.family == STOMSFEM_FAMILY_FEATURES) {
      if (!s.feature_map || s.nfeat < 0 || s.nfeat > 1024 || s.nxi < s.nfeat)
        return pfail(STOMSFEM_EINVAL, w + "bad feature family");
    } else {
      return pfail(STOMSFEM_EINVAL, w + "unknown coefficient family");
    }
  }
  auto* p = new stomsfem_plan();
  hipGetDevice(&p->device);
  p->stages.assign(stages, stages + nstage);
  p->group_of.resize(nstage);
  for (int i = 0; i < nstage; ++i) {
    const stomsfem_stage& s = stages[i];
    int gi = -1;
    for (size_t k = 0; k < p->groups.size(); ++k)
      if (p->groups[k].m == s.m && p->groups[k].ncx == s.ncx) gi = (int)k;
    if (gi < 0) {
      p->groups.emplace_back();
      gi = (int)p->groups.size() - 1;
      p->groups[gi].m = s.m;
      p->groups[gi].ncx = s.ncx;
      p->groups[gi].ncy = s.ncy;
    }
    p->group_of[i] = gi;
    p->groups[gi].stages.push_back(i);
  }
  hipError_t e = hipSuccess;
  for (auto& g : p->groups) {
    size_t a_bytes = 0, nmax = 0;
    for (int i : g.stages) {
      const stomsfem_stage& s = p->stages[i];
      const size_t elt = s.a_dtype == STOMSFEM_F32 ? 4 : 8;
      const size_t nf = (size_t)s.ncx * s.m;
      a_bytes = std::max(a_bytes, elt * (size_t)s.nsamples * nf * nf);
      nmax = std::max(nmax, (size_t)s.nsamples);
    }
    const size_t M = (size_t)g.ncx * g.ncy, nU = (size_t)(g.ncx - 1) * (g.ncy - 1);
    if (e == hipSuccess) e = hipMalloc(&g.a, a_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&g.S, sizeof(double) * nmax * M * 10);
    if (e == hipSuccess) e = hipMalloc((void**)&g.status, sizeof(int32_t) * nmax * M);
    if (e == hipSuccess) e = hipMalloc((void**)&g.cstatus, sizeof(int32_t) * nmax);
    if (e == hipSuccess) e = hipMalloc((void**)&g.work, sizeof(double) * (size_t)coarse_work_doubles(g.ncx, g.ncy, nmax));
    if (e == hipSuccess) e = hipMalloc((void**)&g.U, sizeof(double) * nmax * nU);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g.done, hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    plan_release(p);
    return pfail(STOMSFEM_ENOMEM, "plan_create: device allocation failed");
  }
  // whole-plan graph: one branch per H/h group
  e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) e = hipEventRecord(p->fork, p->capture);
  for (auto& g : p->groups) {
    if (e == hipSuccess) e = hipStreamWaitEvent(g.stream, p->fork, 0);
    for (int i : g.stages)
      if (e == hipSuccess) e = enqueue_stage(p, i, g.stream);
    if (e == hipSuccess) e = hipEventRecord(g.done, g.stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->capture, g.done, 0);
  }
  {
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(p->capture, &graph);
    if (e == hipSuccess) e = e2;
    p->g_all = graph;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->x_all, p->g_all, nullptr, nullptr, 0);
  // one graph per stage
  p->g_stage.assign(nstage, nullptr);
  p->x_stage.assign(nstage, nullptr);
  for (int i = 0; i < nstage && e == hipSuccess; ++i) {
    e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = enqueue_stage(p, i, p->capture);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(p->capture, &graph);
    if (e == hipSuccess) e = e2;
    p->g_stage[i] = graph;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->x_stage[i], graph, nullptr, nullptr, 0);
  }
  if (e != hipSuccess) {
    const std::string msg = std::string("plan_create: graph capture failed: ") + hipGetErrorString(e);
    (void)hipGetLastError();
    plan_release(p);
    return pfail(STOMSFEM_EHIP, msg);
  }
  *plan = p;
  return STOMSFEM_OK;
}

int stomsfem_plan_launch(stomsfem_plan* plan, int32_t stage, void* stream) {
  if (!plan) return pfail(STOMSFEM_EINVAL, "plan_launch: NULL plan");
  if (stage < -1 || stage >= (int32_t)plan->stages.size()) return pfail(STOMSFEM_EINVAL, "plan_launch: bad stage");
  hipGraphExec_t x = stage < 0 ? plan->x_all : plan->x_stage[stage];
  const hipError_t e = hipGraphLaunch(x, (hipStream_t)stream);
  if (e != hipSuccess) return pfail(STOMSFEM_EHIP, std::string("plan_launch: ") + hipGetErrorString(e));
  return STOMSFEM_OK;
}

int stomsfem_plan_free(stomsfem_plan* plan) {
  plan_release(plan);
  return STOMSFEM_OK;
}

}  // extern "C"
