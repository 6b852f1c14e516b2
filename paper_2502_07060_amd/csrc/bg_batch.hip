// Batched launches over mixed (field, n, d) groups: bg_batch_run and the
// hipGraph plans bg_batch_plan_*.
//
// Queue form (BG_BATCH_QUEUE).  The groups whose selected kernel is a
// lane-group (runtime-n) kernel are served by one persistent launch per such
// kernel variant instead of one launch per group: the variant's blocks stay
// resident and take (group, point range) tiles from a device work queue, one
// atomic increment per tile, with the groups ordered by cost per point so the
// longest tiles go first.  Register-kernel groups launch as before.  The
// queue needs device memory beyond the inputs and outputs (one counter per
// persistent launch and the table of its groups): bg_batch_run_ex allocates
// it stream-ordered for the call, a plan at creation, and
// bg_batch_run_noalloc uses a fixed device array of the library instead.
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
#include <cstring>
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

__global__ void bg_queue_reset_kernel(uint32_t* next, int count);

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
  int field, n, d;
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
    pr.field = g.field;
    pr.n = g.n;
    pr.d = g.d;
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

// ---------------------------------------------------------------------------
// queue form
// ---------------------------------------------------------------------------
constexpr size_t kCounterStride = 256;  // one counter per 256 bytes
constexpr int kMaxBuckets = 64;

struct QueueBucket {
  const void* fn = nullptr;  // the variant's bg_wide_queue_kernel
  std::vector<QueueGroup> groups;
  uint32_t ntiles = 0;
  unsigned block = 0, grid = 0, shmem = 0;
  size_t table_off = 0;
  int64_t cost = 0;
};

struct QueuePlan {
  std::vector<Prepared> direct;      // launched one kernel per group
  std::vector<QueueBucket> buckets;  // one persistent launch each
  size_t bytes = 0;                  // counters, then the group tables
};

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

int plan_queue(const bg_group* groups, int ngroups, QueuePlan& qp) {
  std::vector<Prepared> work;
  int rc = prepare_all(groups, ngroups, work);
  if (rc != BG_OK) return rc;
  qp = QueuePlan{};
  std::vector<const Variant*> vs;
  std::vector<std::vector<const Prepared*>> members;
  for (const Prepared& w : work) {
    const Variant* v = w.spec.variant;
    if (!(w.spec.generic && v && v->fn_queue && v->lds_per_point)) {
      qp.direct.push_back(w);
      continue;
    }
    size_t b = 0;
    while (b < vs.size() && vs[b] != v) ++b;
    if (b == vs.size()) {
      vs.push_back(v);
      members.emplace_back();
    }
    members[b].push_back(&w);
  }
  if ((int)vs.size() > kMaxBuckets) return BG_ENOTIMPL;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return BG_EHIP;
  size_t off = up256(vs.size() * kCounterStride);
  for (size_t b = 0; b < vs.size(); ++b) {
    const Variant& v = *vs[b];
    QueueBucket qb;
    qb.fn = v.fn_queue;
    size_t per = 0;
    for (const Prepared* w : members[b]) per = std::max<size_t>(per, v.lds_per_point(w->spec.N));
    int P = wide_points_per_block(v, per);
    while (P > 1 && (size_t)P * per + kQueueLdsHeader > (size_t)max_lds_per_block()) --P;
    qb.block = (unsigned)(P * v.L);
    qb.shmem = (unsigned)(P * per + kQueueLdsHeader);
    if (qb.shmem > (unsigned)max_lds_per_block()) return BG_ENOTIMPL;
    if (qb.shmem > 65536) {
      static std::mutex mu;
      std::lock_guard<std::mutex> lk(mu);
      (void)hipFuncSetAttribute(qb.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)qb.shmem);
    }
    // the groups by cost per point, longest first
    std::vector<const Prepared*> ms = members[b];
    std::stable_sort(ms.begin(), ms.end(), [](const Prepared* a, const Prepared* c) {
      return work_per_point(a->field, a->n, a->d) > work_per_point(c->field, c->n, c->d);
    });
    uint64_t tiles = 0;
    for (const Prepared* w : ms) {
      QueueGroup g;
      g.args = w->spec.args;
      g.N = w->spec.N;
      g.first_tile = (uint32_t)tiles;
      qb.groups.push_back(g);
      tiles += (uint64_t)((w->spec.args.npts + P - 1) / P);
      qb.cost += w->cost;
    }
    if (tiles >= 0xFFFFFFFFull - 0x10000000ull) return BG_EINVAL;  // every block's last increment stays below 2^32
    qb.ntiles = (uint32_t)tiles;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, qb.fn, (int)qb.block, qb.shmem) != hipSuccess ||
        per_cu <= 0)
      return BG_EHIP;
    qb.grid = (unsigned)std::min<uint64_t>((uint64_t)per_cu * cus, tiles);
    qb.table_off = off;
    off = up256(off + qb.groups.size() * sizeof(QueueGroup));
    qp.buckets.push_back(std::move(qb));
  }
  qp.bytes = qp.buckets.empty() ? 0 : off;
  return BG_OK;
}

// the group tables as they lie in the device buffer (from the first table on)
std::vector<unsigned char> queue_tables(const QueuePlan& qp) {
  std::vector<unsigned char> h;
  if (qp.buckets.empty()) return h;
  const size_t base = qp.buckets.front().table_off;
  h.assign(qp.bytes - base, 0);
  for (const QueueBucket& qb : qp.buckets)
    std::memcpy(h.data() + (qb.table_off - base), qb.groups.data(), qb.groups.size() * sizeof(QueueGroup));
  return h;
}

int launch_bucket(const QueueBucket& qb, unsigned char* buf, int b, hipStream_t st) {
  const QueueGroup* groups = reinterpret_cast<const QueueGroup*>(buf + qb.table_off);
  uint32_t* next = reinterpret_cast<uint32_t*>(buf + (size_t)b * kCounterStride);
  int ng = (int)qb.groups.size();
  uint32_t nt = qb.ntiles;
  void* args[] = {&groups, &ng, &nt, &next};
  return hipLaunchKernel(qb.fn, dim3(qb.grid), dim3(qb.block), args, qb.shmem, st) == hipSuccess ? BG_OK : BG_EHIP;
}

// copy the tables into buf and zero the counters (a kernel, not a memset, so
// that the same order also holds inside graphs)
int stage_queue(const QueuePlan& qp, unsigned char* buf, hipStream_t st) {
  if (qp.buckets.empty()) return BG_OK;
  const std::vector<unsigned char> h = queue_tables(qp);
  if (hipMemcpyAsync(buf + qp.buckets.front().table_off, h.data(), h.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return BG_EHIP;
  hipLaunchKernelGGL(bg_queue_reset_kernel, dim3(1), dim3(kMaxBuckets), 0, st, reinterpret_cast<uint32_t*>(buf),
                     (int)qp.buckets.size());
  return hipGetLastError() == hipSuccess ? BG_OK : BG_EHIP;
}

}  // namespace

__global__ void bg_queue_reset_kernel(uint32_t* next, int count) {
  const int i = (int)threadIdx.x;
  if (i < count) next[(size_t)i * (kCounterStride / sizeof(uint32_t))] = 0u;
}

}  // namespace bg

namespace bg {
namespace {

// One launch unit of a run: a direct kernel or a persistent bucket, with its
// estimated cost for the stream balance.
struct Unit {
  const Prepared* direct = nullptr;
  int bucket = -1;
  int64_t cost = 0;
};

std::vector<Unit> units_of(const QueuePlan& qp) {
  std::vector<Unit> u;
  for (const Prepared& w : qp.direct) u.push_back(Unit{&w, -1, w.cost});
  for (size_t b = 0; b < qp.buckets.size(); ++b) u.push_back(Unit{nullptr, (int)b, qp.buckets[b].cost});
  std::stable_sort(u.begin(), u.end(), [](const Unit& a, const Unit& c) { return a.cost > c.cost; });
  return u;
}

int launch_unit(Unit& u, QueuePlan& qp, unsigned char* buf, hipStream_t st) {
  if (u.direct) return enqueue(const_cast<Prepared*>(u.direct)->spec, st);
  return launch_bucket(qp.buckets[u.bucket], buf, u.bucket, st);
}

// units spread over the internal streams (longest first, least loaded
// stream), forked from and joined back to the caller's stream
int run_units(std::vector<Unit>& units, QueuePlan& qp, unsigned char* buf, hipStream_t caller) {
  if (units.empty()) return BG_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceStreams* ds = device_streams();
  if (!ds) return BG_EHIP;
  const int used = std::min<int>(kStreams, (int)units.size());
  if (hipEventRecord(ds->fork, caller) != hipSuccess) return BG_EHIP;
  for (int i = 0; i < used; ++i)
    if (hipStreamWaitEvent(ds->s[i], ds->fork, 0) != hipSuccess) return BG_EHIP;
  int64_t load[kStreams] = {0};
  int rc = BG_OK;
  for (Unit& u : units) {
    int best = 0;
    for (int i = 1; i < used; ++i)
      if (load[i] < load[best]) best = i;
    load[best] += u.cost;
    rc = launch_unit(u, qp, buf, ds->s[best]);
    if (rc != BG_OK) break;
  }
  // join even after a failed launch, so the caller's stream never races ahead
  for (int i = 0; i < used; ++i) {
    if (hipEventRecord(ds->join[i], ds->s[i]) != hipSuccess) return BG_EHIP;
    if (hipStreamWaitEvent(caller, ds->join[i], 0) != hipSuccess) return BG_EHIP;
  }
  return rc;
}

// ---- the fixed device array of bg_batch_run_noalloc ------------------------
// Counters and group tables of one call; each GPU the library runs on holds
// its own copy until the process ends.  Host code must not use the array's
// name as an address: its device address comes from hipGetSymbolAddress,
// once per device.
constexpr size_t kQueueScratchBytes = 256 * 1024;
__device__ __align__(256) unsigned char scratch[kQueueScratchBytes];

std::mutex g_scratch_mu;
std::vector<unsigned char*> g_scratch_ptr;  // per device, null until resolved

unsigned char* scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace bg

struct bg_batch_plan {
  std::vector<bg::Prepared> launches;  // default form
  bg::QueuePlan queue;                 // queue form
  bool use_queue = false;
  unsigned char* buf = nullptr;        // queue form: counters and group tables
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

int bg_batch_run(const bg_group* groups, int ngroups, void* hip_stream) {
  bg::QueuePlan qp;
  const int rc = bg::prepare_all(groups, ngroups, qp.direct);
  if (rc != BG_OK) return rc;
  std::vector<bg::Unit> units = bg::units_of(qp);
  return bg::run_units(units, qp, nullptr, static_cast<hipStream_t>(hip_stream));
}

int bg_batch_run_ex(const bg_group* groups, int ngroups, int flags, void* hip_stream) {
  if (flags & ~BG_BATCH_QUEUE) return BG_EINVAL;
  if (!(flags & BG_BATCH_QUEUE)) return bg_batch_run(groups, ngroups, hip_stream);
  bg::QueuePlan qp;
  int rc = bg::plan_queue(groups, ngroups, qp);
  if (rc != BG_OK) return rc;
  hipStream_t caller = static_cast<hipStream_t>(hip_stream);
  unsigned char* buf = nullptr;
  if (qp.bytes) {
    if (hipMallocAsync(reinterpret_cast<void**>(&buf), qp.bytes, caller) != hipSuccess) return BG_ENOMEM;
    rc = bg::stage_queue(qp, buf, caller);
  }
  std::vector<bg::Unit> units = bg::units_of(qp);
  if (rc == BG_OK) rc = bg::run_units(units, qp, buf, caller);
  if (buf && hipFreeAsync(buf, caller) != hipSuccess && rc == BG_OK) rc = BG_EHIP;
  return rc;
}

int bg_batch_run_noalloc(const bg_group* groups, int ngroups, void* hip_stream) {
  bg::QueuePlan qp;
  int rc = bg::plan_queue(groups, ngroups, qp);
  if (rc != BG_OK) return rc;
  if (qp.bytes > bg::kQueueScratchBytes) return BG_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  unsigned char* buf = nullptr;
  if (qp.bytes) {
    buf = bg::scratch_ptr();
    if (!buf) return BG_EHIP;
    rc = bg::stage_queue(qp, buf, st);
  }
  // everything on the caller's stream (no internal streams to create)
  std::vector<bg::Unit> units = bg::units_of(qp);
  for (size_t i = 0; rc == BG_OK && i < units.size(); ++i) rc = bg::launch_unit(units[i], qp, buf, st);
  return rc;
}

int bg_batch_plan_create_ex(const bg_group* groups, int ngroups, int flags, bg_batch_plan** plan) {
  if (!plan) return BG_EINVAL;
  *plan = nullptr;
  if (flags & ~BG_BATCH_QUEUE) return BG_EINVAL;
  auto* pl = new bg_batch_plan;
  pl->use_queue = (flags & BG_BATCH_QUEUE) != 0;
  int rc = pl->use_queue ? bg::plan_queue(groups, ngroups, pl->queue) : bg::prepare_all(groups, ngroups, pl->launches);
  if (rc == BG_OK && hipGraphCreate(&pl->graph, 0) != hipSuccess) rc = BG_EHIP;
  auto add_kernel = [&](const void* fn, unsigned grid, unsigned block, unsigned shmem, void** args,
                        const hipGraphNode_t* deps, size_t ndeps) {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(block);
    kp.sharedMemBytes = shmem;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    if (hipGraphAddKernelNode(&node, pl->graph, deps, ndeps, &kp) != hipSuccess) rc = BG_EHIP;
  };
  std::vector<bg::Prepared>& direct = pl->use_queue ? pl->queue.direct : pl->launches;
  for (size_t i = 0; rc == BG_OK && i < direct.size(); ++i) {
    bg::LaunchSpec& sp = direct[i].spec;
    void* args_reg[] = {&sp.args};
    void* args_gen[] = {&sp.args, &sp.N};
    add_kernel(sp.fn, sp.grid, sp.block, sp.shmem, sp.generic ? args_gen : args_reg, nullptr, 0);
  }
  if (rc == BG_OK && pl->use_queue && pl->queue.bytes) {
    // the tables are written once here; each replay zeroes the counters with
    // a kernel node that the persistent launches depend on
    if (hipMalloc(reinterpret_cast<void**>(&pl->buf), pl->queue.bytes) != hipSuccess) rc = BG_ENOMEM;
    if (rc == BG_OK) {
      const std::vector<unsigned char> h = bg::queue_tables(pl->queue);
      if (hipMemcpy(pl->buf + pl->queue.buckets.front().table_off, h.data(), h.size(), hipMemcpyHostToDevice) !=
          hipSuccess)
        rc = BG_EHIP;
    }
    hipGraphNode_t reset{};
    if (rc == BG_OK) {
      uint32_t* next = reinterpret_cast<uint32_t*>(pl->buf);
      int count = (int)pl->queue.buckets.size();
      void* args[] = {&next, &count};
      hipKernelNodeParams kp{};
      kp.func = reinterpret_cast<void*>(&bg::bg_queue_reset_kernel);
      kp.gridDim = dim3(1);
      kp.blockDim = dim3(bg::kMaxBuckets);
      kp.sharedMemBytes = 0;
      kp.kernelParams = args;
      kp.extra = nullptr;
      if (hipGraphAddKernelNode(&reset, pl->graph, nullptr, 0, &kp) != hipSuccess) rc = BG_EHIP;
    }
    for (size_t b = 0; rc == BG_OK && b < pl->queue.buckets.size(); ++b) {
      const bg::QueueBucket& qb = pl->queue.buckets[b];
      const bg::QueueGroup* g = reinterpret_cast<const bg::QueueGroup*>(pl->buf + qb.table_off);
      uint32_t* next = reinterpret_cast<uint32_t*>(pl->buf + b * bg::kCounterStride);
      int ng = (int)qb.groups.size();
      uint32_t nt = qb.ntiles;
      void* args[] = {&g, &ng, &nt, &next};
      add_kernel(qb.fn, qb.grid, qb.block, qb.shmem, args, &reset, 1);
    }
  }
  if (rc == BG_OK && hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess) rc = BG_EHIP;
  if (rc != BG_OK) {
    bg_batch_plan_destroy(pl);
    return rc;
  }
  *plan = pl;
  return BG_OK;
}

int bg_batch_plan_create(const bg_group* groups, int ngroups, bg_batch_plan** plan) {
  return bg_batch_plan_create_ex(groups, ngroups, 0, plan);
}

int bg_batch_plan_launch(bg_batch_plan* plan, void* hip_stream) {
  if (!plan) return BG_EINVAL;
  if (plan->launches.empty() && plan->queue.direct.empty() && plan->queue.buckets.empty()) return BG_OK;
  return hipGraphLaunch(plan->exec, static_cast<hipStream_t>(hip_stream)) == hipSuccess ? BG_OK : BG_EHIP;
}

int bg_batch_plan_destroy(bg_batch_plan* plan) {
  if (!plan) return BG_OK;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->buf) (void)hipFree(plan->buf);
  delete plan;
  return BG_OK;
}

}  // extern "C"
