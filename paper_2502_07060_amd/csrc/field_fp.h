// Z_p arithmetic for odd primes p < 2^31 on gfx950 (paper Sec. 3: p < 2^31,
// exact arithmetic, division by the modular inverse).
//
// Representation.  Signed Montgomery form with R = 2^32 (Montgomery 1985):
// a residue x is held as an int32 v with v = x R (mod p), balanced,
// |v| <= h = (p-1)/2.  Products of two such values are below h^2 < 2^60 in
// magnitude, so an int64 accumulator holds 7 of them without overflow.
//
// REDC (signed form): for |T| < p 2^31,
//     t = (int32)(T * pinv mod 2^32),  U = (T - t p) / 2^32   (exact division),
// gives U = T R^-1 (mod p) with |U| < p; one balancing step brings it to
// [-h, h].
//
// Fold: T = hi 2^32 + lo (hi signed, lo in [0, 2^32)) is congruent to
// hi * c32 + lo with c32 = 2^32 mod p (balanced, |c32| <= h); for any int64 T
// the folded value is below 2^31 h + 2^32 <= p 2^30 + 2^32 < p 2^31 (p >= 5),
// so fold-then-REDC is valid for every accumulator, and after a fold five more
// products still fit: 2^61 + 2^32 + 5 * 2^60 < 2^63.
//
// Inputs are interpreted as Montgomery forms themselves (no conversion on
// load): a canonical input x is read as the value x R^-1.  The amplitude is
// homogeneous of degree 4 - n in the momenta and n in the polarisations, so
// the computed value is M R^-4 in Montgomery form, i.e. the stored result is
// M R^-3; one REDC against R^4 mod p on output restores M exactly.
#pragma once

#include "bg_common.h"

namespace bg {

struct FpConst {
  int32_t p;      // the prime
  int32_t h;      // (p - 1) / 2
  uint32_t pinv;  // p^-1 mod 2^32
  int32_t c32;    // 2^32 mod p, balanced        (R in Montgomery form / R)
  int32_t r4;     // R^4 mod p, balanced         (output fix-up factor)
  int32_t two;    // 2 R mod p, balanced           (the constant 2, Montgomery form)
  int32_t inv2;   // 2^-1 R mod p, balanced        (the constant 1/2, Montgomery form)
  int32_t one;    // R mod p, balanced             (the constant 1, Montgomery form)
};

__device__ __forceinline__ int64_t mul64(int32_t a, int32_t b) { return (int64_t)a * (int64_t)b; }

__device__ __forceinline__ int64_t mad64(int32_t a, int32_t b, int64_t c) { return (int64_t)a * (int64_t)b + c; }

// x in (-p, p) -> [-h, h]
__device__ __forceinline__ int32_t fp_balance(int32_t x, const FpConst& F) {
  x = (x > F.h) ? x - F.p : x;
  x = (x < -F.h) ? x + F.p : x;
  return x;
}

// T congruent, |result| < 2^31 h + 2^32
__device__ __forceinline__ int64_t fp_fold(int64_t T, const FpConst& F) {
  int32_t hi = (int32_t)(T >> 32);
  uint32_t lo = (uint32_t)T;
  return mad64(hi, F.c32, (int64_t)lo);
}

// |T| < p 2^31  ->  T R^-1 mod p in (-p, p)
__device__ __forceinline__ int32_t fp_redc_raw(int64_t T, const FpConst& F) {
  int32_t t = (int32_t)((uint32_t)T * F.pinv);
  return (int32_t)((T - mul64(t, F.p)) >> 32);
}

__device__ __forceinline__ int32_t fp_redc(int64_t T, const FpConst& F) {
  return fp_balance(fp_redc_raw(T, F), F);
}

// Montgomery product of balanced values -> balanced
__device__ __forceinline__ int32_t fp_mul(int32_t a, int32_t b, const FpConst& F) {
  return fp_redc(mul64(a, b), F);
}

// balanced a + b, a - b
__device__ __forceinline__ int32_t fp_add(int32_t a, int32_t b, const FpConst& F) {
  return fp_balance(a + b, F);  // |a + b| <= 2h = p - 1 < p
}
__device__ __forceinline__ int32_t fp_sub(int32_t a, int32_t b, const FpConst& F) {
  return fp_balance(a - b, F);
}

// canonical input residue x in [0, p) -> balanced representative
__device__ __forceinline__ int32_t fp_from_canonical(uint32_t x, const FpConst& F) {
  int32_t v = (int32_t)x;
  return v > F.h ? v - F.p : v;
}

__device__ __forceinline__ uint32_t fp_to_canonical(int32_t v, const FpConst& F) {
  return (uint32_t)(v < 0 ? v + F.p : v);
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
