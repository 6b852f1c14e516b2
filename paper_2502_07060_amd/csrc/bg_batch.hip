// Batched launches over mixed (field, n, d) groups: bg_batch_run and the
// hipGraph plans bg_batch_plan_*.
//
// Every group runs the kernel variant selected for its (field, n, d) (the
// autotuner's pin, else the default).  Groups are ordered longest first by
// estimated work and spread over a few internal streams (greedy, least loaded
// first), forked from and joined back to the caller's stream, so small groups
// overlap the tails of large ones.  A plan records the same set of launches
// once as a graph of independent kernel nodes; launching it is one
// hipGraphLaunch however many groups it holds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "bg.h"
#include "bg_registry.h"

namespace bg {

int validate_group(const bg_group& g) {
  if (g.field != BG_FIELD_C128 && g.field != BG_FIELD_FP) return BG_EINVAL;
  if (g.n < 3 || g.n > BG_MAX_N || g.d < 1 || g.d > BG_MAX_D) return BG_EDOMAIN;
  if (g.npts < 0) return BG_EINVAL;
  if (g.field == BG_FIELD_FP && (g.p < 3 || g.p >= 0x80000000u || !is_prime_u32(g.p))) return BG_ENOTPRIME;
  if (g.npts > 0 && (g.ld < g.npts || !g.momenta || !g.pols || !g.out)) return BG_EINVAL;
  return BG_OK;
}

namespace {

constexpr int kStreams = 4;

int64_t work_per_point(int field, int n, int d) {
  const int64_t c3 = (int64_t)n * (n - 1) * (n - 2) / 6;
  const int64_t c4 = c3 * (n - 3) / 4;
  const int64_t R = (int64_t)(n - 1) * (n - 2) / 2 - 1;
  const int64_t W = (int64_t)d * (6 * c3 + 4 * c4 + 2 * R + 1);
  return field == FIELD_C128 ? 2 * W : W;  // a complex multiply-add costs about two F_p ones
}

struct Prepared {
  LaunchSpec spec;
  int64_t cost;
};

int prepare_all(const bg_group* groups, int ngroups, std::vector<Prepared>& out) {
  if (ngroups < 0 || (ngroups > 0 && !groups)) return BG_EINVAL;
  for (int i = 0; i < ngroups; ++i) {
    const int rc = validate_group(groups[i]);
    if (rc != BG_OK) return rc;
  }
  out.clear();
  for (int i = 0; i < ngroups; ++i) {
    const bg_group& g = groups[i];
    if (g.npts == 0) continue;
    Prepared pr;
    FpConst k{};
    if (g.field == BG_FIELD_FP) k = make_fp_const(g.p);
    const int rc = prepare(g.field, g.n, g.d, g.npts, g.ld, g.momenta, g.pols, g.out, g.status, k, pr.spec);
    if (rc != BG_OK) return rc;
    pr.cost = g.npts * work_per_point(g.field, g.n, g.d) * (pr.spec.generic ? (pr.spec.lanes == 1 ? 6 : 2) : 1);
    out.push_back(pr);
  }
  std::stable_sort(out.begin(), out.end(), [](const Prepared& a, const Prepared& b) { return a.cost > b.cost; });
  return BG_OK;
}

// per-device internal streams and events (default priority)
struct DeviceStreams {
  hipStream_t s[kStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kStreams] = {};
  bool ok = false;
};

std::mutex g_mu;
std::vector<DeviceStreams> g_dev;

DeviceStreams* device_streams() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  DeviceStreams& ds = g_dev[dev];
  if (!ds.ok) {
    for (int i = 0; i < kStreams; ++i) {
      if (hipStreamCreateWithFlags(&ds.s[i], hipStreamNonBlocking) != hipSuccess) return nullptr;
      if (hipEventCreateWithFlags(&ds.join[i], hipEventDisableTiming) != hipSuccess) return nullptr;
    }
    if (hipEventCreateWithFlags(&ds.fork, hipEventDisableTiming) != hipSuccess) return nullptr;
    ds.ok = true;
  }
  return &ds;
}

}  // namespace
}  // namespace bg

struct bg_batch_plan {
  std::vector<bg::Prepared> launches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

int bg_batch_run(const bg_group* groups, int ngroups, void* hip_stream) {
  std::vector<bg::Prepared> work;
  int rc = bg::prepare_all(groups, ngroups, work);
  if (rc != BG_OK || work.empty()) return rc;
  hipStream_t caller = static_cast<hipStream_t>(hip_stream);
  std::lock_guard<std::mutex> lk(bg::g_mu);
  bg::DeviceStreams* ds = bg::device_streams();
  if (!ds) return BG_EHIP;
  const int used = std::min<int>(bg::kStreams, (int)work.size());
  if (hipEventRecord(ds->fork, caller) != hipSuccess) return BG_EHIP;
  for (int i = 0; i < used; ++i)
    if (hipStreamWaitEvent(ds->s[i], ds->fork, 0) != hipSuccess) return BG_EHIP;
  int64_t load[bg::kStreams] = {0};
  for (auto& w : work) {
    int best = 0;
    for (int i = 1; i < used; ++i)
      if (load[i] < load[best]) best = i;
    load[best] += w.cost;
    rc = bg::enqueue(w.spec, ds->s[best]);
    if (rc != BG_OK) break;
  }
  // join even after a failed launch, so the caller's stream never races ahead
  for (int i = 0; i < used; ++i) {
    if (hipEventRecord(ds->join[i], ds->s[i]) != hipSuccess) return BG_EHIP;
    if (hipStreamWaitEvent(caller, ds->join[i], 0) != hipSuccess) return BG_EHIP;
  }
  return rc;
}

int bg_batch_plan_create(const bg_group* groups, int ngroups, bg_batch_plan** plan) {
  if (!plan) return BG_EINVAL;
  *plan = nullptr;
  auto* pl = new bg_batch_plan;
  int rc = bg::prepare_all(groups, ngroups, pl->launches);
  if (rc == BG_OK && hipGraphCreate(&pl->graph, 0) != hipSuccess) rc = BG_EHIP;
  for (size_t i = 0; rc == BG_OK && i < pl->launches.size(); ++i) {
    bg::LaunchSpec& sp = pl->launches[i].spec;
    void* args_reg[] = {&sp.args};
    void* args_gen[] = {&sp.args, &sp.N};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(sp.fn);
    kp.gridDim = dim3(sp.grid);
    kp.blockDim = dim3(sp.block);
    kp.sharedMemBytes = sp.shmem;
    kp.kernelParams = sp.generic ? args_gen : args_reg;
    kp.extra = nullptr;
    hipGraphNode_t node;
    if (hipGraphAddKernelNode(&node, pl->graph, nullptr, 0, &kp) != hipSuccess) rc = BG_EHIP;
  }
  if (rc == BG_OK && hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess) rc = BG_EHIP;
  if (rc != BG_OK) {
    bg_batch_plan_destroy(pl);
    return rc;
  }
  *plan = pl;
  return BG_OK;
}

int bg_batch_plan_launch(bg_batch_plan* plan, void* hip_stream) {
  if (!plan) return BG_EINVAL;
  if (plan->launches.empty()) return BG_OK;
  return hipGraphLaunch(plan->exec, static_cast<hipStream_t>(hip_stream)) == hipSuccess ? BG_OK : BG_EHIP;
}

int bg_batch_plan_destroy(bg_batch_plan* plan) {
  if (!plan) return BG_OK;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
  return BG_OK;
}

}  // extern "C"
