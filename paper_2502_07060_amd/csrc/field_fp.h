// Z_p arithmetic for odd primes p < 2^31 on gfx950 (paper Sec. 3: p < 2^31,
// exact arithmetic, division by the modular inverse).
//
// Representation.  Signed Montgomery form (Montgomery 1985) with R = 2^64,
// reduced in two 32-bit steps: a residue x is held as an int32 v with
// v = x R (mod p), balanced, |v| <= h = (p-1)/2.  Products of two such
// values are below h^2 < 2^60 in magnitude, so an int64 accumulator holds
// seven of them without overflow.
//
// REDC2.  For |T| < 2^62:
//     t1 = (int32)(T * pinv mod 2^32),  T1 = (T - t1 p) / 2^32,
//     t2 = (int32)(T1 * pinv mod 2^32), T2 = (T1 - t2 p) / 2^32,
// with pinv = p^-1 mod 2^32 and both divisions exact.  |T - t1 p| < 2^63 and
// |T1| < (2^62 + 2^31 p) / 2^32 < 2^31, so T1 is an int32; then
// |T2| < (2^31 + 2^31 p) / 2^32 = h + 1, so T2 = T R^-1 (mod p) comes out
// balanced with no compare-and-select step.
//
// Fold.  T = hi 2^32 + lo (hi signed, lo in [0, 2^32)) is congruent to
// hi * c32 + lo with c32 = 2^32 mod p balanced; for any int64 T the folded
// value is below 2^31 h + 2^32 < 2^61 + 2^32, which REDC2 accepts, and after
// a fold five more products still fit in int64.
//
// Inputs are read as Montgomery forms themselves (no conversion on load): a
// canonical input x stands for x R^-1.  The amplitude is homogeneous of degree
// 4 - n in the momenta and n in the polarisations, so the computed value is
// M R^-4 in Montgomery form, i.e. the stored result is M R^-3; one REDC2
// against R^4 mod p on output restores M exactly.
#pragma once

#include "bg_common.h"

namespace bg {

struct FpConst {
  int32_t p;      // the prime
  int32_t h;      // (p - 1) / 2
  uint32_t pinv;  // p^-1 mod 2^32
  int32_t negp;   // -p
  int32_t c32;    // 2^32 mod p, balanced  (fold constant)
  int32_t c64;    // 2^64 mod p = R mod p, balanced: the constant 1 in Montgomery form,
                  // and the factor that lifts a Montgomery value into a product accumulator
  int32_t r4;     // R^4 mod p, balanced   (output fix-up factor)
  int32_t r4s;    // R^4 2^-32 mod p, balanced (output fix-up of the register kernel, whose
                  // accumulators carry the extra 2^32 of lazily reduced scalars)
  int32_t r3;     // R^3 mod p, balanced   (fix-up of a root current, degree n - 1 in eps)
  int32_t r3s;    // R^3 2^-32 mod p, balanced (the same in the register kernel)
  int32_t two;    // 2 R mod p, balanced   (the constant 2, Montgomery form)
  int32_t two32;  // 2^33 mod p, balanced  (2 R 2^-32: the constant 2 with an extra 2^-32)
  int32_t inv2;   // 2^-1 R mod p, balanced (the constant 1/2, Montgomery form)
  int32_t one;    // R mod p (= c64)
};

__device__ __forceinline__ int64_t mul64(int32_t a, int32_t b) { return (int64_t)a * (int64_t)b; }

__device__ __forceinline__ int64_t mad64(int32_t a, int32_t b, int64_t c) { return (int64_t)a * (int64_t)b + c; }

// T congruent, |result| < 2^31 h + 2^32.  Formed as T + hi c32 (modulo 2^64)
// with hi then taken off the high word: one multiply-add into T itself and
// one 32-bit subtraction, no zero-extended copy of lo.
__device__ __forceinline__ int64_t fp_fold(int64_t T, const FpConst& F) {
  const int32_t hi = (int32_t)(T >> 32);
  u32x2 r = __builtin_bit_cast(u32x2, (uint64_t)T + (uint64_t)mul64(hi, F.c32));
  r.y -= (uint32_t)hi;
  return (int64_t)__builtin_bit_cast(uint64_t, r);
}

// one 32-bit REDC step: |T| < 2^61 + 2^32  ->  T 2^-32 mod p with
// |result| < 2^30 + 2^29 + 1 (an int32, not balanced)
__device__ __forceinline__ int32_t fp_redc1(int64_t T, const FpConst& F) {
  const int32_t t1 = (int32_t)((uint32_t)T * F.pinv);
  return (int32_t)(mad64(t1, F.negp, T) >> 32);
}

// |T| < 2^62  ->  T R^-1 mod p, balanced
__device__ __forceinline__ int32_t fp_redc2(int64_t T, const FpConst& F) {
  const int32_t t1 = (int32_t)((uint32_t)T * F.pinv);
  const int32_t T1 = (int32_t)(mad64(t1, F.negp, T) >> 32);
  const int32_t t2 = (int32_t)((uint32_t)T1 * F.pinv);
  return (int32_t)(mad64(t2, F.negp, (int64_t)T1) >> 32);
}

// Montgomery product of balanced values -> balanced
__device__ __forceinline__ int32_t fp_mul(int32_t a, int32_t b, const FpConst& F) {
  return fp_redc2(mul64(a, b), F);
}

// any |x| < 2^31 -> the balanced representative of x (x c64 R^-1 = x)
__device__ __forceinline__ int32_t fp_norm(int32_t x, const FpConst& F) {
  return fp_redc2(mul64(x, F.c64), F);
}

__device__ __forceinline__ int32_t fp_add(int32_t a, int32_t b, const FpConst& F) {
  return fp_norm(a + b, F);  // |a + b| <= 2h < 2^31
}
__device__ __forceinline__ int32_t fp_sub(int32_t a, int32_t b, const FpConst& F) {
  return fp_norm(a - b, F);
}

// canonical input residue x in [0, p) -> balanced representative
__device__ __forceinline__ int32_t fp_from_canonical(uint32_t x, const FpConst& F) {
  const int32_t v = (int32_t)x;
  return v - (((F.h - v) >> 31) & F.p);
}

__device__ __forceinline__ uint32_t fp_to_canonical(int32_t v, const FpConst& F) {
  return (uint32_t)(v + ((v >> 31) & F.p));
}

// a^e for a balanced Montgomery value; e is uniform across the wave, so the
// branch on its bits does not diverge.
__device__ __forceinline__ int32_t fp_pow(int32_t a, uint32_t e, const FpConst& F) {
  int32_t r = F.one;
  int top = 31 - __builtin_clz(e);
  for (int b = top; b >= 0; --b) {
    r = fp_mul(r, r, F);
    if ((e >> b) & 1u) r = fp_mul(r, a, F);
  }
  return r;
}

}  // namespace bg
