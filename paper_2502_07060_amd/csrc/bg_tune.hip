// Autotuner: times every compiled kernel variant for a (field, n, d) on
// synthetic device inputs and pins the fastest (see bg_autotune in bg.h).
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "bg.h"
#include "bg_registry.h"

namespace bg {
bool is_prime_u32(uint32_t n);
}

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  // splitmix64 finaliser (Steele, Lea, Flood 2014)
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// uniform residues in [0, p) (p > 0) or, for p == 0, complex values with
// parts in [-1, 1); count = number of 32-bit (F_p) or complex (C) elements
__global__ void fill_kernel(void* dst, int64_t count, uint32_t p, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t r = mix64(seed ^ (uint64_t)i);
  if (p) {
    static_cast<uint32_t*>(dst)[i] = (uint32_t)((r >> 32) % p);
  } else {
    const double a = (double)(r >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    const double b = (double)(mix64(r) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    static_cast<double2*>(dst)[i] = make_double2(a, b);
  }
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" int bg_autotune_metric(int metric, int field, int n, int d, uint32_t p, int64_t npts, int reps,
                                  double* ms_out, int cap, void* hip_stream) {
  if (metric != BG_METRIC_MOSTLY_MINUS && metric != BG_METRIC_ALTERNATING) return BG_EINVAL;
  if (field != BG_FIELD_C128 && field != BG_FIELD_FP) return BG_EINVAL;
  if (n < 3 || n > BG_MAX_N || d < 1 || d > BG_MAX_D) return BG_EDOMAIN;
  if (npts <= 0 || reps <= 0) return BG_EINVAL;
  if (field == BG_FIELD_FP && (p < 3 || p >= 0x80000000u || !bg::is_prime_u32(p))) return BG_ENOTPRIME;
  if (field == BG_FIELD_FP && metric == BG_METRIC_ALTERNATING && p % 4 != 1) return BG_EDOMAIN;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int count = bg_variants(field, n, d, nullptr, 0);
  if (count <= 0) return count < 0 ? count : BG_ENOTIMPL;
  std::vector<bg_variant_info> vs(count);
  bg_variants(field, n, d, vs.data(), count);
  // the current pin of this metric, restored if tuning fails (a pinned
  // variant stays pinned; an unpinned (field, n, d) stays on its default)
  const int prev = bg::pinned_index(field, n, d, metric);

  const size_t elem = field == BG_FIELD_FP ? 4 : 16;
  const int64_t nelem = (int64_t)n * d * npts;
  DevBuf mom, pol, out, sta;
  if (hipMalloc(&mom.p, nelem * elem) != hipSuccess || hipMalloc(&pol.p, nelem * elem) != hipSuccess ||
      hipMalloc(&out.p, npts * elem) != hipSuccess || hipMalloc(&sta.p, npts) != hipSuccess)
    return BG_ENOMEM;
  const uint32_t fp = field == BG_FIELD_FP ? p : 0;
  const int64_t blocks = (nelem + 255) / 256;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, mom.p, nelem, fp, 0x1234ull);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, pol.p, nelem, fp, 0x5678ull);
  if (hipGetLastError() != hipSuccess) return BG_EHIP;

  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return BG_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return BG_EHIP;
  }
  auto run = [&]() {
    if (field == BG_FIELD_FP)
      return bg_amplitudes_fp_metric(metric, n, d, npts, npts, p, (const uint32_t*)mom.p, (const uint32_t*)pol.p,
                                     (uint32_t*)out.p, (uint8_t*)sta.p, st);
    return bg_amplitudes_c128_metric(metric, n, d, npts, npts, (const double*)mom.p, (const double*)pol.p,
                                     (double*)out.p, (uint8_t*)sta.p, st);
  };
  int rc = BG_OK;
  // time of one launch of variant k, averaged over reps after a warm-up
  auto time_variant = [&](int k, double& per) {
    bg::select_variant(metric, field, n, d, vs[k].index);
    rc = run();  // warm-up
    float ms = 0.f;
    if (rc == BG_OK && hipEventRecord(e0, st) != hipSuccess) rc = BG_EHIP;
    for (int r = 0; r < reps && rc == BG_OK; ++r) rc = run();
    if (rc == BG_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = BG_EHIP;
    per = rc == BG_OK ? (double)ms / reps : -1.0;
  };
  std::vector<double> per(count, 1e300);
  for (int k = 0; k < count && rc == BG_OK; ++k) time_variant(k, per[k]);
  // variants within 5 % of the fastest are timed again, in turns, three more
  // times, each keeping its best: one pass cannot separate kernels that close
  // (clocks and the order of the pass move single timings by a few percent)
  if (rc == BG_OK) {
    const double first = *std::min_element(per.begin(), per.end());
    std::vector<int> close;
    for (int k = 0; k < count; ++k)
      if (per[k] <= 1.05 * first) close.push_back(k);
    for (int round = 0; round < 3 && close.size() > 1 && rc == BG_OK; ++round)
      for (int k : close) {
        double t = 0.0;
        time_variant(k, t);
        if (rc != BG_OK) break;
        per[k] = std::min(per[k], t);
      }
  }
  int best = -1;
  double best_ms = 1e300;
  for (int k = 0; k < count && rc == BG_OK; ++k) {
    if (ms_out && k < cap) ms_out[k] = per[k];
    if (per[k] < best_ms) {
      best_ms = per[k];
      best = vs[k].index;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != BG_OK || best < 0) {
    bg::select_variant(metric, field, n, d, prev);
    return rc != BG_OK ? rc : BG_EHIP;
  }
  bg::select_variant(metric, field, n, d, best);
  return best;
}

extern "C" int bg_autotune(int field, int n, int d, uint32_t p, int64_t npts, int reps, double* ms_out,
                           int cap, void* hip_stream) {
  return bg_autotune_metric(BG_METRIC_MOSTLY_MINUS, field, n, d, p, npts, reps, ms_out, cap, hip_stream);
}

// Selections as text, one line per pinned (field, n, d, metric):
//   field n d lanes comps_per_lane lds_tables generic padded max_d metric
// Lines name kernels by their shape, so a file stays valid across builds that
// register kernels in another order; lines with no matching kernel are
// skipped, and a line without the metric column is a mostly-minus pin.
extern "C" int bg_tune_save(const char* path) {
  if (!path) return BG_EINVAL;
  FILE* f = fopen(path, "w");
  if (!f) return BG_EINVAL;
  fprintf(f, "# field n d lanes comps_per_lane lds_tables generic padded max_d metric\n");
  bg_variant_info vs[128];
  for (int field = 0; field <= 1; ++field)
    for (int n = 3; n <= BG_MAX_N; ++n)
      for (int d = 1; d <= BG_MAX_D; ++d) {
        const int c = std::min(128, bg_variants(field, n, d, vs, 128));
        for (int metric : {BG_METRIC_MOSTLY_MINUS, BG_METRIC_ALTERNATING}) {
          const int idx = bg::pinned_index(field, n, d, metric);
          for (int k = 0; k < c && idx >= 0; ++k)
            if (vs[k].index == idx)
              fprintf(f, "%d %d %d %d %d %d %d %d %d %d\n", field, n, d, vs[k].lanes, vs[k].comps_per_lane,
                      vs[k].lds_tables, vs[k].generic, vs[k].padded, vs[k].max_d, metric);
        }
      }
  fclose(f);
  return BG_OK;
}

extern "C" int bg_tune_load(const char* path) {
  if (!path) return BG_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return BG_EINVAL;
  char line[256];
  int applied = 0;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    int field, n, d, lanes, dl, lt, gen, pad = 0, maxd = 0, metric = BG_METRIC_MOSTLY_MINUS;
    if (sscanf(line, "%d %d %d %d %d %d %d %d %d %d", &field, &n, &d, &lanes, &dl, &lt, &gen, &pad, &maxd,
               &metric) < 7)
      continue;
    bg_variant_info vs[128];
    const int c = bg_variants(field, n, d, vs, 128);
    for (int k = 0; k < std::min(c, 128); ++k)
      if (vs[k].lanes == lanes && vs[k].comps_per_lane == dl && vs[k].lds_tables == lt && vs[k].generic == gen &&
          vs[k].padded == pad && (maxd == 0 || vs[k].max_d == maxd)) {
        if (bg::select_variant(metric, field, n, d, vs[k].index) == BG_OK) ++applied;
        break;
      }
  }
  fclose(f);
  return applied;
}
