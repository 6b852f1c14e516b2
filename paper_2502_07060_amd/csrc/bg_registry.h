// Registry of compiled kernel variants.  Each instantiation unit registers
// its kernels at load time; the launch layer picks one per (field, n, d).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "bg.h"
#include "bg_kernel.h"

namespace bg {

enum : int { FIELD_C128 = 0, FIELD_FP = 1 };

struct Variant {
  int field;
  int N;          // n - 1 (0 for the runtime-n kernels)
  int DL;         // components per lane (DMAX for the runtime-n kernels)
  int L;          // lanes per point (runtime-n: 1 = one point per lane, G = lanes sharing a point)
  int block;      // threads per block (0: chosen at launch)
  bool generic;   // runtime-n kernel with LDS tables
  bool lds_tables;  // register kernel with per-point tables in LDS
  int waves;        // minimum waves per SIMD the register allocation allows
  const void* fn;
  unsigned (*lds_per_point)(int N) = nullptr;  // runtime-n kernels: LDS bytes per point
  bool padded = false;  // lane-group kernel whose table rows are padded to an odd number of 16-byte units
  int split = 1;        // lane-group kernel: lanes per work item (DL / split components each)
  // Z_p register kernel compiled for the small-fold-constant schedule (primes
  // with |2^32 mod p| <= 2^22); the launch takes it instead of fn for those
  const void* fn_sc = nullptr;
  // lane-group kernel: its persistent work-queue form (bg_wide_queue_kernel)
  const void* fn_queue = nullptr;
};

// |2^32 mod p| (balanced) <= 2^22: the small-fold-constant schedule applies
inline bool fp_small_fold(const FpConst& k) { return k.c32 >= -(1 << 22) && k.c32 <= (1 << 22); }

std::vector<Variant>& registry();
// pins per metric (BG_METRIC_*): pinned_index is -1 where none
bool is_pinned(int field, int n, int d, int metric = BG_METRIC_MOSTLY_MINUS);
int pinned_index(int field, int n, int d, int metric);
int select_variant(int metric, int field, int n, int d, int index);

// A fully prepared launch of one (field, n, d) batch: kernel, grid and the
// argument block (kept alive by the owner, e.g. a graph plan).
struct LaunchSpec {
  const Variant* variant = nullptr;
  const void* fn = nullptr;
  unsigned grid = 0, block = 0, shmem = 0;
  bool generic = false;  // runtime-n kernel (takes N as a second argument)
  int lanes = 1;         // lanes per point
  int N = 0;
  LaunchArgs args;
};

FpConst make_fp_const(uint32_t p);
// a square root of -1 mod p (p = 1 mod 4) times R = 2^64, balanced
int32_t fp_sqrt_minus_one_mont(uint32_t p);
bool is_prime_u32(uint32_t n);
// force: the variant to launch instead of the one selected for (field, n, d)
int prepare(int field, int n, int d, int64_t npts, int64_t ld, const void* momenta, const void* pols,
            void* out, uint8_t* status, const FpConst& fp, LaunchSpec& spec, const Variant* force = nullptr);
int enqueue(LaunchSpec& spec, hipStream_t stream);
// lane-group launches: points per block for LDS bytes per point `per`, the
// one that keeps the most points resident per CU
int wide_points_per_block(const Variant& v, size_t per);
int max_lds_per_block();
// argument checks of one bg_group (field, ranges, prime, pointers)
int validate_group(const bg_group& g);

struct Registrar {
  explicit Registrar(const Variant& v) { registry().push_back(v); }
};

// LDS bytes per point of a runtime-n kernel (one instantiation per layout)
template <class Layout>
unsigned generic_lds_bytes(int N) {
  return (unsigned)Layout::bytes_per_point(N);
}
template <class Layout>
unsigned wide_lds_bytes(int N) {
  return Layout::offsets(N).total;
}

}  // namespace bg

#define BG_CAT2(a, b) a##b
#define BG_CAT(a, b) BG_CAT2(a, b)

// register-resident kernel for field FLD (FpField / C128Field), N, DL, L,
// with the per-point tables in LDS when LT is true, W waves per SIMD
#define BG_REGISTER_RECURSION(FIELDTAG, FLD, N_, DL_, L_, LT_, W_)                                      \
  namespace bg {                                                                                        \
  template __global__ void bg_recursion_kernel<FLD<DL_, L_>, N_, DL_, L_, 256, LT_, W_>(LaunchArgs);   \
  static Registrar BG_CAT(reg_, __COUNTER__)(Variant{                                                   \
      FIELDTAG, N_, DL_, L_, 256, false, LT_, W_,                                                       \
      reinterpret_cast<const void*>(&bg_recursion_kernel<FLD<DL_, L_>, N_, DL_, L_, 256, LT_, W_>)});   \
  }

// the same for Z_p: both reduction schedules, selected per launch by the prime
#define BG_REGISTER_RECURSION_FP(N_, DL_, L_, LT_, W_)                                                       \
  namespace bg {                                                                                             \
  template __global__ void bg_recursion_kernel<FpField<DL_, L_, false>, N_, DL_, L_, 256, LT_, W_>(LaunchArgs); \
  template __global__ void bg_recursion_kernel<FpField<DL_, L_, true>, N_, DL_, L_, 256, LT_, W_>(LaunchArgs);  \
  static Registrar BG_CAT(reg_, __COUNTER__)(Variant{                                                        \
      FIELD_FP, N_, DL_, L_, 256, false, LT_, W_,                                                            \
      reinterpret_cast<const void*>(&bg_recursion_kernel<FpField<DL_, L_, false>, N_, DL_, L_, 256, LT_, W_>), \
      nullptr, false, 1,                                                                                     \
      reinterpret_cast<const void*>(&bg_recursion_kernel<FpField<DL_, L_, true>, N_, DL_, L_, 256, LT_, W_>)}); \
  }

#define BG_REGISTER_GENERIC(FIELDTAG, FLD, DMAX_)                                               \
  namespace bg {                                                                                \
  template __global__ void bg_generic_kernel<FLD<DMAX_, 1>, DMAX_>(LaunchArgs, int);            \
  static Registrar BG_CAT(reg_, __COUNTER__)(Variant{                                           \
      FIELDTAG, 0, DMAX_, 1, 0, true, true, 1,                                                  \
      reinterpret_cast<const void*>(&bg_generic_kernel<FLD<DMAX_, 1>, DMAX_>),                  \
      &generic_lds_bytes<GenericLayout<FLD<DMAX_, 1>, DMAX_>>});                                \
  }

// runtime-n kernel with G work items sharing each point's tables, LC lanes per
// item (PAD: odd row stride)
#define BG_REGISTER_WIDE(FIELDTAG, FLD, DMAX_, G_, PAD_, LC_)                                               \
  namespace bg {                                                                                            \
  template __global__ void bg_wide_kernel<FLD<DMAX_ / LC_, LC_>, DMAX_, G_, PAD_>(LaunchArgs, int);         \
  template __global__ void bg_wide_queue_kernel<FLD<DMAX_ / LC_, LC_>, DMAX_, G_, PAD_>(                    \
      const QueueGroup*, int, uint32_t, uint32_t*);                                                         \
  static Registrar BG_CAT(reg_, __COUNTER__)(Variant{                                                       \
      FIELDTAG, 0, DMAX_, G_ * LC_, 0, true, true, 1,                                                       \
      reinterpret_cast<const void*>(&bg_wide_kernel<FLD<DMAX_ / LC_, LC_>, DMAX_, G_, PAD_>),               \
      &wide_lds_bytes<WideLayout<FLD<DMAX_ / LC_, LC_>, DMAX_, G_, PAD_>>, PAD_, LC_, nullptr,              \
      reinterpret_cast<const void*>(&bg_wide_queue_kernel<FLD<DMAX_ / LC_, LC_>, DMAX_, G_, PAD_>)});       \
  }
