// C-ABI entry points of libbg_mi355x.so (declared in include/bg.h).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "bg.h"
#include "bg_wide.h"
#include "bg_registry.h"

namespace bg {

std::vector<Variant>& registry() {
  static std::vector<Variant> r;
  return r;
}

// ---------------------------------------------------------------------------
// primes and Montgomery constants
// ---------------------------------------------------------------------------
static uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = (unsigned __int128)r * a % m;
    a = (unsigned __int128)a * a % m;
    e >>= 1;
  }
  return r;
}

// Deterministic Miller-Rabin for n < 4,759,123,141 with bases 2, 7, 61
// (Jaeschke 1993).
bool is_prime_u32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t sp : {2u, 3u, 5u, 7u, 11u, 13u, 61u})
    if (n % sp == 0) return n == sp;
  uint32_t dd = n - 1;
  int r = 0;
  while ((dd & 1) == 0) { dd >>= 1; ++r; }
  for (uint32_t base : {2u, 7u, 61u}) {
    uint64_t x = powmod(base, dd, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r; ++i) {
      x = (unsigned __int128)x * x % n;
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

static int32_t balanced(uint64_t x, uint32_t p) {
  x %= p;
  return x > (p - 1) / 2 ? (int32_t)((int64_t)x - p) : (int32_t)x;
}

FpConst make_fp_const(uint32_t p) {
  FpConst k;
  k.p = (int32_t)p;
  k.h = (int32_t)((p - 1) / 2);
  uint32_t inv = p;  // Newton iteration for p^-1 mod 2^32 (p odd)
  for (int i = 0; i < 5; ++i) inv *= 2u - p * inv;
  k.pinv = inv;
  k.negp = -(int32_t)p;
  const uint64_t c32 = (uint64_t(1) << 32) % p;
  const uint64_t R = (unsigned __int128)c32 * c32 % p;  // 2^64 mod p
  k.c32 = balanced(c32, p);
  k.c64 = balanced(R, p);
  k.one = k.c64;
  k.two = balanced(2 * R, p);
  k.two32 = balanced(2 * c32, p);  // 2^33 mod p
  k.inv2 = balanced((unsigned __int128)R * ((p + 1) / 2) % p, p);
  const uint64_t R2 = (unsigned __int128)R * R % p;
  k.r4 = balanced((unsigned __int128)R2 * R2 % p, p);
  // 2^-32 mod p = (2^32 mod p)^(p-2)
  const uint64_t inv32 = powmod(c32, p - 2, p);
  k.r4s = balanced((unsigned __int128)((unsigned __int128)R2 * R2 % p) * inv32 % p, p);
  k.r3 = balanced((unsigned __int128)R2 * R % p, p);
  k.r3s = balanced((unsigned __int128)((unsigned __int128)R2 * R % p) * inv32 % p, p);
  return k;
}

// a square root of -1 mod p (p = 1 mod 4) in Montgomery form: g^((p-1)/4) R
// for the smallest quadratic non-residue g, balanced
int32_t fp_sqrt_minus_one_mont(uint32_t p) {
  uint64_t g = 2;
  while (powmod(g, (p - 1) / 2, p) != p - 1) ++g;
  const uint64_t i = powmod(g, (p - 1) / 4, p);
  const uint64_t c32 = (uint64_t(1) << 32) % p;
  const uint64_t R = (unsigned __int128)c32 * c32 % p;
  return balanced((unsigned __int128)i * R % p, p);
}

// ---------------------------------------------------------------------------
// variant choice
// ---------------------------------------------------------------------------
// Default lanes per point, from timings on gfx950 at n = 8 (F_p d = 6: two
// lanes 0.70 ms vs one lane 0.80 ms per 2^20 points; complex d = 4: two lanes
// 0.92 ms vs four 1.10 ms); bg_autotune measures the rest.
static int preferred_lanes(int field, int N, int d) {
  (void)field;
  (void)N;
  (void)d;
  return 2;
}

static bool fits(const Variant& v, int field, int n, int d) {
  if (v.field != field) return false;
  if (v.generic) return v.DL >= d;
  return v.N == n - 1 && v.DL * v.L >= d;
}

// selections, per metric: launches in the alternating metric have pins of
// their own (a kernel's two metric forms can compile to code of different
// speed), and fall back to the mostly-minus choice
struct Pin {
  int field, n, d, metric, index;
};
static std::mutex g_pin_mu;
static std::vector<Pin> g_pins;

static int pinned(int field, int n, int d, int metric) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  for (const Pin& p : g_pins)
    if (p.field == field && p.n == n && p.d == d && p.metric == metric) return p.index;
  return -1;
}

bool is_pinned(int field, int n, int d, int metric) { return pinned(field, n, d, metric) >= 0; }

int pinned_index(int field, int n, int d, int metric) { return pinned(field, n, d, metric); }

int select_variant(int metric, int field, int n, int d, int index) {
  if (field != BG_FIELD_C128 && field != BG_FIELD_FP) return BG_EINVAL;
  if (metric != BG_METRIC_MOSTLY_MINUS && metric != BG_METRIC_ALTERNATING) return BG_EINVAL;
  if (n < 3 || n > BG_MAX_N || d < 1 || d > BG_MAX_D) return BG_EDOMAIN;
  if (index >= 0 && (index >= (int)registry().size() || !fits(registry()[index], field, n, d)))
    return BG_EINVAL;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  for (auto it = g_pins.begin(); it != g_pins.end(); ++it)
    if (it->field == field && it->n == n && it->d == d && it->metric == metric) {
      g_pins.erase(it);
      break;
    }
  if (index >= 0) g_pins.push_back({field, n, d, metric, index});
  return BG_OK;
}

const Variant* default_variant(int field, int n, int d);

// a wide kernel keeps at least 512 lanes (8 waves) busy per CU at this N
static bool best_fills(const Variant* v, int N) {
  const unsigned per = v->lds_per_point ? v->lds_per_point(N) : 0;
  return per && (long)(max_lds_per_block() / per) * v->L >= 512;
}

const Variant* choose_variant(int field, int n, int d) {
  const int idx = pinned(field, n, d, BG_METRIC_MOSTLY_MINUS);
  if (idx >= 0 && idx < (int)registry().size() && fits(registry()[idx], field, n, d))
    return &registry()[idx];
  return default_variant(field, n, d);
}

const Variant* default_variant(int field, int n, int d) {
  const int N = n - 1;
  const int L = preferred_lanes(field, N, d);
  const int need = (d + L - 1) / L;
  const Variant* best = nullptr;
  for (const Variant& v : registry()) {
    if (v.generic || v.field != field || v.N != N || v.L != L || v.DL < need) continue;
    if (best && best->DL == v.DL && !v.lds_tables) continue;  // prefer the LDS-table form on ties
    if (!best || v.DL < best->DL) best = &v;
  }
  if (best) return best;
  for (const Variant& v : registry()) {  // any register kernel that fits, fewest padded slots
    if (v.generic || !fits(v, field, n, d)) continue;
    if (!best || v.DL * v.L < best->DL * best->L || (v.DL * v.L == best->DL * best->L && v.L < best->L))
      best = &v;
  }
  if (best) return best;
  // runtime-n kernels: the smallest DMAX that covers d; among those the
  // lane-sharing (wide) form whose resident points fill a CU with the fewest
  // lanes per point, else the one-point-per-lane form
  int dmax = 0;
  for (const Variant& v : registry())
    if (v.generic && v.field == field && v.DL >= d && (!dmax || v.DL < dmax)) dmax = v.DL;
  for (const Variant& v : registry()) {
    if (!v.generic || v.field != field || v.DL != dmax || v.L == 1) continue;
    const unsigned per = v.lds_per_point ? v.lds_per_point(N) : 0;
    const long resident = per ? (long)(max_lds_per_block() / per) * v.L : 0;
    const bool fills = resident >= 512;
    if (!best || (fills && (best->L > v.L || !best_fills(best, N))) || (!fills && !best_fills(best, N) && v.L > best->L))
      best = &v;
    else if (v.L == best->L && v.padded && !best->padded)
      best = &v;  // padded rows are compiled only where they avoid bank conflicts
  }
  if (best) return best;
  for (const Variant& v : registry())
    if (v.generic && v.field == field && v.DL == dmax) return &v;
  return nullptr;
}

int max_lds_per_block() {
  static std::once_flag once;
  static int v = 65536;
  std::call_once(once, [] {
    int dev = 0, val = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&val, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        val > 0)
      v = val;
  });
  return v;
}

int prepare(int field, int n, int d, int64_t npts, int64_t ld, const void* momenta, const void* pols,
            void* out, uint8_t* status, const FpConst& fp, LaunchSpec& spec, const Variant* force) {
  const Variant* v = force ? force : choose_variant(field, n, d);
  if (!v) return BG_ENOTIMPL;
  LaunchArgs& a = spec.args;
  a.momenta = momenta;
  a.pols = pols;
  a.out = out;
  a.status = status;
  a.npts = npts;
  a.ld = ld;
  a.d = d;
  a.fp = fp;
  a.metric = BG_METRIC_MOSTLY_MINUS;
  a.ialt = fp.one;  // the mostly-minus factor; launch() sets i R for the alternating metric
  a.cur = nullptr;
  spec.variant = v;
  spec.fn = (field == FIELD_FP && v->fn_sc && fp_small_fold(fp)) ? v->fn_sc : v->fn;
  spec.generic = v->generic;
  spec.lanes = v->L;
  spec.N = n - 1;
  if (!v->generic) {
    const int64_t threads = npts * v->L;
    const int64_t blocks = (threads + v->block - 1) / v->block;
    if (blocks > 0x7FFFFFFF) return BG_EINVAL;
    spec.grid = (unsigned)blocks;
    spec.block = (unsigned)v->block;
    spec.shmem = 0;
    return BG_OK;
  }
  const size_t per = v->lds_per_point ? v->lds_per_point(n - 1) : 0;
  const int maxlds = max_lds_per_block();
  if (per == 0 || per > (size_t)maxlds) return BG_ENOTIMPL;
  int P;  // points per block
  if (v->L == 1) {
    P = (int)std::min<size_t>(256, (size_t)maxlds / per);
    if (P >= 64) P = P / 64 * 64;
  } else {
    P = wide_points_per_block(*v, per);
  }
  if (P < 1) return BG_ENOTIMPL;
  const size_t shmem = per * P;
  if (shmem > 65536) {
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    (void)hipFuncSetAttribute(v->fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  }
  const int64_t blocks = (npts + P - 1) / P;
  if (blocks > 0x7FFFFFFF) return BG_EINVAL;
  spec.grid = (unsigned)blocks;
  spec.block = (unsigned)(P * v->L);
  spec.shmem = (unsigned)shmem;
  return BG_OK;
}

int wide_points_per_block(const Variant& v, size_t per) {
  // G lanes per point: the block size whose blocks hold the most points per
  // CU (LDS and 32 wave slots per CU), among blocks of whole wavefronts when
  // one fits: a block of fewer lanes than a wave still takes a wave slot and
  // issues every instruction for 64 lanes, so half-full waves halve the work
  // done per instruction
  const int maxlds = max_lds_per_block();
  const int pmax = std::min<int>(256 / v.L, (int)((size_t)maxlds / per));
  const int step = v.L < 64 ? 64 / v.L : 1;  // points per whole wave
  const int first = step <= pmax ? step : 1;
  const int inc = step <= pmax ? step : 1;
  int P = 1;
  long bestres = 0;
  for (int c = first; c <= pmax; c += inc) {
    const long waves = ((long)c * v.L + 63) / 64;
    const long blocks = std::min<long>((long)maxlds / ((long)c * (long)per), 32 / waves);
    const long res = blocks * c;
    if (res > bestres || (res == bestres && c > P)) { bestres = res; P = c; }
  }
  return P;
}

int enqueue(LaunchSpec& spec, hipStream_t stream) {
  void* args_reg[] = {&spec.args};
  void* args_gen[] = {&spec.args, &spec.N};
  hipError_t e = hipLaunchKernel(spec.fn, dim3(spec.grid), dim3(spec.block),
                                 spec.generic ? args_gen : args_reg, spec.shmem, stream);
  return e == hipSuccess ? BG_OK : BG_EHIP;
}

// Without a pin of their own, alternating-metric launches take the
// mostly-minus choice, except that a one-lane F_p register kernel is replaced
// by the two-lane one of the same (n, d): the one-lane kernels' alternating
// body runs about twice as long as their mostly-minus body (the compiler waits
// for each of its loads before issuing the next; n = 8, d = 6: 0.97 against
// 0.47 ms per 2^20 points), the two-lane kernel's within a few percent of its
// own.
static const Variant* alternating_variant(const Variant* v, int field, int n, int d) {
  if (!v || field != FIELD_FP || v->generic || v->L != 1) return v;
  const Variant* best = nullptr;
  for (const Variant& w : registry()) {
    if (w.generic || w.field != field || w.N != n - 1 || w.L != 2 || w.DL * 2 < d) continue;
    if (!best || w.DL < best->DL || (w.DL == best->DL && w.lds_tables && !best->lds_tables)) best = &w;
  }
  return best ? best : v;
}

int launch(int field, int n, int d, int64_t npts, int64_t ld, const void* momenta, const void* pols,
           void* out, uint8_t* status, const FpConst& fp, hipStream_t stream, int metric = BG_METRIC_MOSTLY_MINUS) {
  LaunchSpec spec;
  const Variant* force = nullptr;
  if (metric == BG_METRIC_ALTERNATING) {
    const int idx = pinned(field, n, d, BG_METRIC_ALTERNATING);
    force = idx >= 0 ? &registry()[idx] : alternating_variant(choose_variant(field, n, d), field, n, d);
  }
  const int rc = prepare(field, n, d, npts, ld, momenta, pols, out, status, fp, spec, force);
  if (rc != BG_OK) return rc;
  spec.args.metric = metric;
  if (metric == BG_METRIC_ALTERNATING && field == FIELD_FP) spec.args.ialt = fp_sqrt_minus_one_mont((uint32_t)fp.p);
  return enqueue(spec, stream);
}

static int check_common(int n, int d, int64_t npts, int64_t ld) {
  if (n < 3 || n > BG_MAX_N || d < 1 || d > BG_MAX_D) return BG_EDOMAIN;
  if (npts < 0) return BG_EINVAL;
  (void)ld;
  return BG_OK;
}

static int check_buffers(int64_t npts, int64_t ld, const void* m, const void* e, const void* o) {
  if (ld < npts || !m || !e || !o) return BG_EINVAL;
  return BG_OK;
}

}  // namespace bg

extern "C" {

int bg_amplitudes_c128_metric(int metric, int n, int d, int64_t npts, int64_t ld, const double* momenta,
                              const double* pols, double* out, uint8_t* status, void* hip_stream) {
  if (metric != BG_METRIC_MOSTLY_MINUS && metric != BG_METRIC_ALTERNATING) return BG_EINVAL;
  int rc = bg::check_common(n, d, npts, ld);
  if (rc != BG_OK) return rc;
  if (npts == 0) return BG_OK;
  rc = bg::check_buffers(npts, ld, momenta, pols, out);
  if (rc != BG_OK) return rc;
  bg::FpConst none;
  memset(&none, 0, sizeof(none));
  return bg::launch(bg::FIELD_C128, n, d, npts, ld, momenta, pols, out, status, none,
                    static_cast<hipStream_t>(hip_stream), metric);
}

int bg_amplitudes_c128(int n, int d, int64_t npts, int64_t ld, const double* momenta,
                       const double* pols, double* out, uint8_t* status, void* hip_stream) {
  return bg_amplitudes_c128_metric(BG_METRIC_MOSTLY_MINUS, n, d, npts, ld, momenta, pols, out, status,
                                   hip_stream);
}

int bg_amplitudes_fp_metric(int metric, int n, int d, int64_t npts, int64_t ld, uint32_t p,
                            const uint32_t* momenta, const uint32_t* pols, uint32_t* out, uint8_t* status,
                            void* hip_stream) {
  if (metric != BG_METRIC_MOSTLY_MINUS && metric != BG_METRIC_ALTERNATING) return BG_EINVAL;
  int rc = bg::check_common(n, d, npts, ld);
  if (rc != BG_OK) return rc;
  if (p < 3 || p >= 0x80000000u || !bg::is_prime_u32(p)) return BG_ENOTPRIME;
  if (metric == BG_METRIC_ALTERNATING && p % 4 != 1) return BG_EDOMAIN;  // needs a square root of -1
  if (npts == 0) return BG_OK;
  rc = bg::check_buffers(npts, ld, momenta, pols, out);
  if (rc != BG_OK) return rc;
  const bg::FpConst k = bg::make_fp_const(p);
  return bg::launch(bg::FIELD_FP, n, d, npts, ld, momenta, pols, out, status, k,
                    static_cast<hipStream_t>(hip_stream), metric);
}

int bg_amplitudes_fp(int n, int d, int64_t npts, int64_t ld, uint32_t p, const uint32_t* momenta,
                     const uint32_t* pols, uint32_t* out, uint8_t* status, void* hip_stream) {
  return bg_amplitudes_fp_metric(BG_METRIC_MOSTLY_MINUS, n, d, npts, ld, p, momenta, pols, out, status,
                                 hip_stream);
}

// root current K([1..n-1]) instead of M: same preparation, `cur` in place of `out`
static int launch_currents(int field, int n, int d, int64_t npts, int64_t ld, const void* momenta,
                           const void* pols, void* cur, uint8_t* status, const bg::FpConst& fp,
                           hipStream_t stream) {
  bg::LaunchSpec spec;
  const int rc = bg::prepare(field, n, d, npts, ld, momenta, pols, nullptr, status, fp, spec);
  if (rc != BG_OK) return rc;
  spec.args.cur = cur;
  return bg::enqueue(spec, stream);
}

int bg_currents_c128(int n, int d, int64_t npts, int64_t ld, const double* momenta, const double* pols,
                     double* cur, uint8_t* status, void* hip_stream) {
  int rc = bg::check_common(n, d, npts, ld);
  if (rc != BG_OK) return rc;
  if (npts == 0) return BG_OK;
  rc = bg::check_buffers(npts, ld, momenta, pols, cur);
  if (rc != BG_OK) return rc;
  bg::FpConst none;
  memset(&none, 0, sizeof(none));
  return launch_currents(bg::FIELD_C128, n, d, npts, ld, momenta, pols, cur, status, none,
                         static_cast<hipStream_t>(hip_stream));
}

int bg_currents_fp(int n, int d, int64_t npts, int64_t ld, uint32_t p, const uint32_t* momenta,
                   const uint32_t* pols, uint32_t* cur, uint8_t* status, void* hip_stream) {
  int rc = bg::check_common(n, d, npts, ld);
  if (rc != BG_OK) return rc;
  if (p < 3 || p >= 0x80000000u || !bg::is_prime_u32(p)) return BG_ENOTPRIME;
  if (npts == 0) return BG_OK;
  rc = bg::check_buffers(npts, ld, momenta, pols, cur);
  if (rc != BG_OK) return rc;
  const bg::FpConst k = bg::make_fp_const(p);
  return launch_currents(bg::FIELD_FP, n, d, npts, ld, momenta, pols, cur, status, k,
                         static_cast<hipStream_t>(hip_stream));
}

int bg_variants(int field, int n, int d, bg_variant_info* out, int cap) {
  if (field != BG_FIELD_C128 && field != BG_FIELD_FP) return BG_EINVAL;
  if (n < 3 || n > BG_MAX_N || d < 1 || d > BG_MAX_D) return BG_EDOMAIN;
  const bg::Variant* cur = bg::choose_variant(field, n, d);
  int count = 0;
  const auto& reg = bg::registry();
  for (int i = 0; i < (int)reg.size(); ++i) {
    if (!bg::fits(reg[i], field, n, d)) continue;
    if (out && count < cap) {
      bg_variant_info& o = out[count];
      o.index = i;
      o.lanes = reg[i].L;
      o.comps_per_lane = reg[i].DL / reg[i].split;
      o.lds_tables = reg[i].lds_tables ? 1 : 0;
      o.generic = reg[i].generic ? 1 : 0;
      o.padded = reg[i].padded ? 1 : 0;
      o.max_d = reg[i].generic ? reg[i].DL : reg[i].DL * reg[i].L;
      o.selected = (&reg[i] == cur) ? 1 : 0;
    }
    ++count;
  }
  return count;
}

int bg_select_variant(int field, int n, int d, int index) {
  return bg::select_variant(BG_METRIC_MOSTLY_MINUS, field, n, d, index);
}

int bg_select_variant_metric(int metric, int field, int n, int d, int index) {
  return bg::select_variant(metric, field, n, d, index);
}

const char* bg_strerror(int code) {
  switch (code) {
    case BG_OK: return "success";
    case BG_EINVAL: return "invalid argument (null pointer, npts < 0 or ld < npts)";
    case BG_EDOMAIN: return "n or d outside the supported range";
    case BG_ENOTPRIME: return "p is not an odd prime below 2^31";
    case BG_EHIP: return "HIP runtime error or kernel launch failure";
    case BG_ENOTIMPL: return "no kernel for this (field, n, d)";
    case BG_ENOMEM: return "request does not fit the memory budget";
    case BG_EBUSY: return "queue full";
    default: return "unknown error code";
  }
}

int bg_version(void) { return 100; }

}  // extern "C"
