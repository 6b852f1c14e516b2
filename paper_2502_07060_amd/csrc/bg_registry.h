// Registry of compiled kernel variants.  Each instantiation unit registers
// its kernels at load time; the launch layer picks one per (field, n, d).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace bg {

enum : int { FIELD_C128 = 0, FIELD_FP = 1 };

struct Variant {
  int field;
  int N;          // n - 1 (0 for the runtime-n generic kernel)
  int DL;         // components per lane (DMAX for the generic kernel)
  int L;          // lanes per point
  int block;      // threads per block
  bool generic;   // runtime-n kernel with LDS tables
  const void* fn;
};

std::vector<Variant>& registry();

struct Registrar {
  explicit Registrar(const Variant& v) { registry().push_back(v); }
};

}  // namespace bg

#define BG_CAT2(a, b) a##b
#define BG_CAT(a, b) BG_CAT2(a, b)

// register-resident kernel for field FLD (FpField / C128Field), N, DL, L
#define BG_REGISTER_RECURSION(FIELDTAG, FLD, N_, DL_, L_)                                       \
  namespace bg {                                                                                \
  template __global__ void bg_recursion_kernel<FLD<DL_, L_>, N_, DL_, L_, 256>(LaunchArgs);    \
  static Registrar BG_CAT(reg_, __COUNTER__)(Variant{                                           \
      FIELDTAG, N_, DL_, L_, 256, false,                                                        \
      reinterpret_cast<const void*>(&bg_recursion_kernel<FLD<DL_, L_>, N_, DL_, L_, 256>)});    \
  }

#define BG_REGISTER_GENERIC(FIELDTAG, FLD, DMAX_)                                               \
  namespace bg {                                                                                \
  template __global__ void bg_generic_kernel<FLD<DMAX_, 1>, DMAX_>(LaunchArgs, int);            \
  static Registrar BG_CAT(reg_, __COUNTER__)(Variant{                                           \
      FIELDTAG, 0, DMAX_, 1, 0, true,                                                           \
      reinterpret_cast<const void*>(&bg_generic_kernel<FLD<DMAX_, 1>, DMAX_>)});                \
  }
