// Field policies used by the recursion kernel.  Each lane holds DL of the d
// Lorentz components of every vector (components mu = s*DL + c for group lane
// s, slot c); the point's L lanes sum dot products over DPP.
//
// Dot products are formed against a "primed" left operand x' = (-x^0, x^1,
// ..., x^{d-1}), so that sum_mu x'_mu y_mu = -(x.y) with uniform signs over
// all slots; every dot product helper therefore returns the NEGATED
// Minkowski product, and the recursion is written with that in mind.
#pragma once

#include "bg_common.h"
#include "field_fp.h"

namespace bg {

// ---------------------------------------------------------------------------
// Z_p, signed balanced Montgomery (see field_fp.h)
// ---------------------------------------------------------------------------
template <int DL, int L>
struct FpField {
  using E = int32_t;  // one component
  using S = int32_t;  // a scalar
  using A = int64_t;  // accumulator of one component
  static constexpr bool exact = true;
  FpConst k;
  bool time_lane;  // group lane 0: slot 0 is mu = 0

  __device__ FpField(const FpConst& c, int s) : k(c), time_lane(s == 0) {}

  __device__ __forceinline__ E prime0(E x) const {
    if constexpr (L == 1) return -x;
    else return time_lane ? -x : x;
  }
  __device__ __forceinline__ E esub(E a, E b) const { return fp_sub(a, b, k); }
  __device__ __forceinline__ E eadd(E a, E b) const { return fp_add(a, b, k); }
  __device__ __forceinline__ S sneg(S a) const { return -a; }
  __device__ __forceinline__ S szero() const { return 0; }
  __device__ __forceinline__ A azero() const { return 0; }

  // Accumulator bounds are tracked in "units" of 2^60 at compile time (every
  // loop here is unrolled): a product of two balanced values is below one
  // unit, a product with a difference of two balanced values below two; a
  // folded accumulator is below two units; an int64 holds up to eight.
  template <int UX>
  __device__ __forceinline__ void acc_dot(A& t, int& u, const E* x, const E* y) const {
#pragma unroll
    for (int c = 0; c < DL; ++c) {
      if (u + UX > 7) {
        t = fp_fold(t, k);
        u = 2;
      }
      t = mad64(x[c], y[c], t);
      u += UX;
    }
  }

  // group-wide sum of lane partials below u units each, then REDC (which
  // needs fewer than four units)
  __device__ __forceinline__ S finish_dot(A t, int u) const {
    if constexpr (L > 1) {
      if (L * u > 7) {
        t = fp_fold(t, k);
        u = 2;
        if (L * u > 7) {  // a second fold leaves below 2^59 + 2^33
          t = fp_fold(t, k);
          u = 1;
        }
      }
      t = group_sum<L>(t, [](A a, A b) { return a + b; },
                       [](auto ctrl, A v) { return (A)dpp_u64<decltype(ctrl)::value>((uint64_t)v); });
      u *= L;
    }
    if (u > 3) t = fp_fold(t, k);
    return fp_redc2(t, k);
  }

  // -(x.y) for primed x (x' slots already carry the time sign); UX = 2 when
  // the slots of x are unreduced differences of two balanced values
  template <int UX = 1>
  __device__ __forceinline__ S ndot(const E* xp, const E* y) const {
    A t = 0;
    int u = 0;
    acc_dot<UX>(t, u, xp, y);
    return finish_dot(t, u);
  }

  // -(x.y) for unprimed x: slot 0 is primed on the fly
  __device__ __forceinline__ S ndot_u(const E* x, const E* y) const {
    E x0[DL];
#pragma unroll
    for (int c = 0; c < DL; ++c) x0[c] = x[c];
    x0[0] = prime0(x[0]);
    return ndot<1>(x0, y);
  }

  // -(x.y) - z  (z a balanced Montgomery value, lifted into the product
  // accumulator by the factor R mod p, added once per group on group lane 0)
  template <int UX = 1>
  __device__ __forceinline__ S ndot_sub(const E* xp, const E* y, S z) const {
    A t = 0;
    int u = 0;
    acc_dot<UX>(t, u, xp, y);
    if (u + 1 > 7) {
      t = fp_fold(t, k);
      u = 2;
    }
    if constexpr (L == 1) t = mad64(-z, k.c64, t);
    else t = mad64(time_lane ? -z : 0, k.c64, t);
    return finish_dot(t, u + 1);
  }

  __device__ __forceinline__ void axpy(A* K, S c, const E* v) const {
#pragma unroll
    for (int i = 0; i < DL; ++i) K[i] = mad64(c, v[i], K[i]);
  }
  __device__ __forceinline__ void fold(A* K) const {
#pragma unroll
    for (int i = 0; i < DL; ++i) K[i] = fp_fold(K[i], k);
  }
  __device__ __forceinline__ E finish(A K) const { return fp_redc2(fp_fold(K, k), k); }
  // finish(K) * c for a c carrying an extra factor 2^-32 (one 32-bit REDC step
  // instead of a full one before the product)
  __device__ __forceinline__ E finish_mul32(A K, S c) const {
    return fp_redc2(mul64(fp_redc1(fp_fold(K, k), k), c), k);
  }
  __device__ __forceinline__ E mul(E x, S c) const { return fp_mul(x, c, k); }
  __device__ __forceinline__ S smul(S a, S b) const { return fp_mul(a, b, k); }
};

// ---------------------------------------------------------------------------
// complex binary64
// ---------------------------------------------------------------------------
struct cplx {
  double re, im;
};

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cneg(cplx a) { return {-a.re, -a.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {__builtin_fma(a.re, b.re, -a.im * b.im), __builtin_fma(a.re, b.im, a.im * b.re)};
}
// acc + a b
__device__ __forceinline__ cplx cmad(cplx a, cplx b, cplx acc) {
  acc.re = __builtin_fma(a.re, b.re, acc.re);
  acc.re = __builtin_fma(-a.im, b.im, acc.re);
  acc.im = __builtin_fma(a.re, b.im, acc.im);
  acc.im = __builtin_fma(a.im, b.re, acc.im);
  return acc;
}

template <int DL, int L>
struct C128Field {
  using E = cplx;
  using S = cplx;
  using A = cplx;
  static constexpr bool exact = false;
  double time_sign;  // -1 on the lane holding mu = 0 (slot 0), +1 elsewhere

  __device__ C128Field(int s) : time_sign((L == 1 || s == 0) ? -1.0 : 1.0) {}

  __device__ __forceinline__ E prime0(E x) const {
    if constexpr (L == 1) return cneg(x);
    else return {x.re * time_sign, x.im * time_sign};
  }
  __device__ __forceinline__ E esub(E a, E b) const { return csub(a, b); }
  __device__ __forceinline__ E eadd(E a, E b) const { return cadd(a, b); }
  __device__ __forceinline__ S sneg(S a) const { return cneg(a); }
  __device__ __forceinline__ S szero() const { return {0.0, 0.0}; }
  __device__ __forceinline__ A azero() const { return {0.0, 0.0}; }

  __device__ __forceinline__ S finish_dot(cplx t) const {
    if constexpr (L > 1) {
      t = group_sum<L>(t, [](cplx a, cplx b) { return cadd(a, b); },
                       [](auto ctrl, cplx v) {
                         constexpr int C = decltype(ctrl)::value;
                         return cplx{dpp_f64<C>(v.re), dpp_f64<C>(v.im)};
                       });
    }
    return t;
  }
  __device__ __forceinline__ S ndot(const E* xp, const E* y) const {
    cplx t = cmul(xp[0], y[0]);
#pragma unroll
    for (int c = 1; c < DL; ++c) t = cmad(xp[c], y[c], t);
    return finish_dot(t);
  }
  __device__ __forceinline__ S ndot_u(const E* x, const E* y) const {
    cplx t = cmul(prime0(x[0]), y[0]);
#pragma unroll
    for (int c = 1; c < DL; ++c) t = cmad(x[c], y[c], t);
    return finish_dot(t);
  }
  __device__ __forceinline__ S ndot_sub(const E* xp, const E* y, S z) const {
    return csub(ndot(xp, y), z);
  }
  __device__ __forceinline__ void axpy(A* K, S c, const E* v) const {
#pragma unroll
    for (int i = 0; i < DL; ++i) K[i] = cmad(c, v[i], K[i]);
  }
  __device__ __forceinline__ void fold(A*) const {}
  __device__ __forceinline__ E finish(A K) const { return K; }
  __device__ __forceinline__ E mul(E x, S c) const { return cmul(x, c); }
  __device__ __forceinline__ S smul(S a, S b) const { return cmul(a, b); }
};

}  // namespace bg
