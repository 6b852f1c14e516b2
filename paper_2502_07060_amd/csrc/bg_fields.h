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
// Two reduction schedules, chosen per launch from the prime:
//
// * general (SC = false): any odd p < 2^31.  Accumulator bounds are tracked
//   at compile time in half-units of 2^59 (an int64 holds 16); a fold leaves
//   up to 2^61 + 2^32, so products are folded in small groups and the
//   register kernel folds its current accumulators at fixed places.
//
// * small fold constant (SC = true): primes whose balanced 2^32 mod p is at
//   most 2^22 in magnitude -- every prime 2^31 - c with c <= 2^21 (the
//   largest primes below 2^31, the usual choice for modular evaluation), and
//   every p < 2^22.  A fold then leaves |hi c32 + lo| <= 2^31 2^22 + 2^32 <
//   2^54, so one fold empties an accumulator almost completely.  Bounds are
//   tracked in units of 2^54 (an int64 holds 511):
//     balanced x balanced             h^2 < 2^60             64
//     unreduced difference x balanced 2h h < 2^61            128
//     folded accumulator              < 2^54                 1
//   and a lazily reduced scalar (one 32-bit REDC step of an input below
//   2 units, 2^55) satisfies |s| <= h + 2^23, so
//     lazy scalar x balanced          < 2^60 + 2^53          65
//     lazy scalar x difference        < 2^61 + 2^54          129
//     lazy scalar x c32 (lift of z)   < 2^53                 1
//   The register kernel then folds a current's accumulator only when the
//   next product would pass 511 units (every loop is unrolled, so the
//   counters are compile-time constants).
template <int DL, int L, bool SC = false>
struct FpField {
  static constexpr int kDL = DL, kL = L;
  static constexpr bool kSC = SC;
  using E = int32_t;  // one component
  using S = int32_t;  // a scalar
  using A = int64_t;  // accumulator of one component
  static constexpr bool exact = true;
  FpConst k;
  bool time_lane;  // group lane 0: slot 0 is mu = 0
  // the factor that lifts a subtracted scalar z into a product accumulator,
  // negated, on group lane 0 only (z is added once per group): by R for a
  // balanced z, by 2^32 for a lazily reduced one
  int32_t zlift64, zlift32;
  // zlift64 and zlift32 again, in registers the compiler cannot see are
  // equal to them: otherwise it rewrites x c + y c as (x + y) c in 64 bits, a
  // multi-instruction 64-bit product instead of two multiply-adds
  int32_t zlift64w, zlift32w;

  __device__ FpField(const FpConst& c, int s)
      : k(c), time_lane(s == 0),
        zlift64((L == 1 || s == 0) ? -c.c64 : 0), zlift32((L == 1 || s == 0) ? -c.c32 : 0),
        zlift64w(zlift64), zlift32w(zlift32) {
    asm volatile("" : "+v"(zlift64w), "+v"(zlift32w));
  }

  __device__ __forceinline__ E prime0(E x) const {
    if constexpr (L == 1) return -x;
    else return time_lane ? -x : x;
  }
  __device__ __forceinline__ E esub(E a, E b) const { return fp_sub(a, b, k); }
  // small fold constant only: |x| <= 2h (an int32 difference of balanced
  // values) -> the same residue with |result| <= h + 2^23, by one product with
  // 2^32 mod p (below 2^53) and one 32-bit REDC step (x c32 2^-32 = x mod p)
  __device__ __forceinline__ E lazy_norm(int32_t x) const {
    static_assert(SC, "needs |2^32 mod p| <= 2^22");
    return fp_redc1(mul64(x, k.c32), k);
  }
  __device__ __forceinline__ E eadd(E a, E b) const { return fp_add(a, b, k); }
  __device__ __forceinline__ S sneg(S a) const { return -a; }
  __device__ __forceinline__ S szero() const { return 0; }
  __device__ __forceinline__ A azero() const { return 0; }

  // Bound bookkeeping.  General schedule: half-units of 2^59, an int64 holds
  // 16 and 15 are used.  A product of two balanced values (|v| <= h < 2^30)
  // is below 2; with one factor an unreduced difference of two balanced
  // values (< 2^31), below 4; with one factor a lazily reduced scalar
  // (|s| < 1.5 2^30 + 1, from one 32-bit REDC step), below 3 (plus 2^30,
  // negligible against the 2^59 kept spare); a folded accumulator is below 4.
  // Small-fold-constant schedule: units of 2^54 (table above).
  static constexpr int kMaxU = SC ? 511 : 15;
  static constexpr int kFoldU = SC ? 1 : 4;     // a folded accumulator
  static constexpr int kLazyIn = SC ? 2 : 4;    // input limit of the lazy 32-bit REDC step
  static constexpr int kRedc2In = SC ? 256 : 8;  // input limit of REDC2 (2^62)
  // product classes, by the template tags the callers pass (UX = 2: balanced
  // slots, UX = 4: unreduced differences; UZ = 2: balanced z lifted by R,
  // UZ = 3: lazy z lifted by 2^32)
  // Small fold constant: the currents themselves are lazily normalised
  // (|J| <= h + 2^23, from two 32-bit REDC steps, see finish_mul32), so
  // UX = 2 counts a product of two such values, (h + 2^23)^2 < 2^60 + 2^55
  // (66 units), and UX = 4 an unreduced difference times one, 2h (h + 2^23)
  // < 2^61 + 2^54 (129); UX = 5 (both operands lazily normalised) is 66 too.
  static constexpr int ux_units(int UX) { return SC ? (UX == 4 ? 129 : 66) : UX; }
  static constexpr int uz_units(int UZ) { return SC ? (UZ == 3 ? 1 : 64) : UZ; }
  // products that enter a current's accumulator (SC schedule only; vectors
  // are currents (|.| <= h + 2^23) or balanced prefix sums)
  static constexpr int kPLazy = 66;       // lazy scalar x current
  static constexpr int kPBal = 65;        // balanced scalar x current
  static constexpr int kPBalDiff = 128;   // balanced scalar x unreduced sum of two balanced values

  template <int UX>
  __device__ __forceinline__ void acc_dot(A& t, int& u, const E* x, const E* y) const {
#pragma unroll
    for (int c = 0; c < DL; ++c) {
      if (u + ux_units(UX) > kMaxU) {
        t = fp_fold(t, k);
        u = kFoldU;
      }
      t = mad64(x[c], y[c], t);
      u += ux_units(UX);
    }
  }

  // group-wide sum of lane partials below u each, then either a full REDC2
  // (balanced result) or, LAZY, one 32-bit REDC step (general: input folded,
  // result |s| < 1.5 2^30 + 1; small fold constant: input below 2^55, result
  // |s| <= h + 2^23) for scalars that only multiply balanced vectors.  A lazy
  // result is the REDC2 one times 2^32 mod p; a caller uses lazy scalars for
  // every term of an accumulator, so the whole accumulator carries the same
  // factor, removed once when it is finished.
  template <bool LAZY>
  __device__ __forceinline__ S finish_dot(A t, int u) const {
    if constexpr (L > 1) {
      if (L * u > kMaxU) {
        t = fp_fold(t, k);
        u = kFoldU;
        if (L * u > kMaxU) {  // general: a second fold leaves below 2^59 + 2^33
          t = fp_fold(t, k);
          u = 2;
        }
      }
      t = group_sum<L>(t, [](A a, A b) { return a + b; },
                       [](auto ctrl, A v) { return (A)dpp_u64<decltype(ctrl)::value>((uint64_t)v); });
      u *= L;
    }
    if constexpr (LAZY) {
      if (u > kLazyIn) t = fp_fold(t, k);
      return fp_redc1(t, k);
    } else {
      if (u >= kRedc2In) t = fp_fold(t, k);
      return fp_redc2(t, k);
    }
  }

  // -(x.y) for primed x (x' slots already carry the time sign); UX = 2 for
  // balanced slots of x, 4 when they are unreduced differences
  template <int UX = 2, bool LAZY = false>
  __device__ __forceinline__ S ndot(const E* xp, const E* y) const {
    A t = 0;
    int u = 0;
    acc_dot<UX>(t, u, xp, y);
    return finish_dot<LAZY>(t, u);
  }

  // -(x.y) for unprimed balanced x: slot 0 is primed on the fly
  template <bool LAZY = false>
  __device__ __forceinline__ S ndot_u(const E* x, const E* y) const {
    E x0[DL];
#pragma unroll
    for (int c = 0; c < DL; ++c) x0[c] = x[c];
    x0[0] = prime0(x[0]);
    return ndot<2, LAZY>(x0, y);
  }

  // -(x.y) - z  (z lifted into the product accumulator, added once per group
  // on group lane 0).  UZ = 2: z balanced, lifted by R mod p; UZ = 3: z a
  // lazily reduced scalar (which carries an extra 2^32), lifted by 2^32 mod p
  template <int UX = 2, int UZ = 2, bool LAZY = false>
  __device__ __forceinline__ S ndot_sub(const E* xp, const E* y, S z) const {
    static_assert(UZ == 2 || UZ == 3, "z is balanced or lazily reduced");
    A t = 0;
    int u = 0;
    acc_dot<UX>(t, u, xp, y);
    if (u + uz_units(UZ) > kMaxU) {
      t = fp_fold(t, k);
      u = kFoldU;
    }
    t = mad64(z, UZ == 3 ? zlift32 : zlift64, t);
    return finish_dot<LAZY>(t, u + uz_units(UZ));
  }

  // -(x.y) - z - w: ndot_sub with a second term w, a balanced scalar lifted
  // like a z of class UW: by 2^32 mod p (UW = 3, w carrying the factor of the
  // lazy scalars) or by R mod p (UW = 2, a plain balanced w)
  template <int UX = 2, int UZ = 2, bool LAZY = false, int UW = 3>
  __device__ __forceinline__ S ndot_sub2(const E* xp, const E* y, S z, S w) const {
    static_assert(UW == 2 || UW == 3, "w is lifted by R or by 2^32");
    static_assert(UZ == 2 || UZ == 3, "z is balanced or lazily reduced");
    A t = 0;
    int u = 0;
    acc_dot<UX>(t, u, xp, y);
    if (u + uz_units(UZ) > kMaxU) {
      t = fp_fold(t, k);
      u = kFoldU;
    }
    t = mad64(z, UZ == 3 ? zlift32 : zlift64, t);
    u += uz_units(UZ);
    if (u + uz_units(UW) > kMaxU) {
      t = fp_fold(t, k);
      u = kFoldU;
    }
    t = mad64(w, UW == 3 ? zlift32w : zlift64w, t);
    return finish_dot<LAZY>(t, u + uz_units(UW));
  }

  __device__ __forceinline__ void axpy(A* K, S c, const E* v) const {
#pragma unroll
    for (int i = 0; i < DL; ++i) K[i] = mad64(c, v[i], K[i]);
  }
  __device__ __forceinline__ void fold(A* K) const {
#pragma unroll
    for (int i = 0; i < DL; ++i) K[i] = fp_fold(K[i], k);
  }

  // Accumulator schedule of the register kernel.  General: the kernel folds
  // at fixed places (fixed_fold) and kaxpy is a plain axpy.  Small fold
  // constant: kaxpy folds only when the product class UP (units of 2^54)
  // would pass the int64 budget, and fixed_fold does nothing.
  template <int UP>
  __device__ __forceinline__ void kaxpy(A* K, int& u, S c, const E* v) const {
    if constexpr (SC) {
      if (u + UP > kMaxU) {
        fold(K);
        u = kFoldU;
      }
      u += UP;
    }
    axpy(K, c, v);
  }
  template <int UP>
  __device__ __forceinline__ void kmad(A& t, int& u, S a, S b) const {
    if constexpr (SC) {
      if (u + UP > kMaxU) {
        t = fp_fold(t, k);
        u = kFoldU;
      }
      u += UP;
    }
    t = mad64(a, b, t);
  }
  __device__ __forceinline__ void fixed_fold(A* K) const {
    if constexpr (!SC) fold(K);
  }

  __device__ __forceinline__ E finish(A K) const { return fp_redc2(fp_fold(K, k), k); }
  // finish(K) * c for a c carrying an extra factor 2^-32 (one 32-bit REDC step
  // instead of a full one before the product).  Small fold constant: the
  // product is finished with one more fold and 32-bit REDC step instead of
  // REDC2 (c then carries 2^-64, see Inverses), leaving |J| <= h + 2^22.
  __device__ __forceinline__ E finish_mul32(A K, S c) const {
    if constexpr (SC) return fp_redc1(fp_fold(mul64(fp_redc1(fp_fold(K, k), k), c), k), k);
    else return fp_redc2(mul64(fp_redc1(fp_fold(K, k), k), c), k);
  }
  // small fold constant: a b 2^-32 mod p for |a|, |b| <= h + 2^23 (a product
  // in the Montgomery domain of 2^32), result |.| <= h + 2^22
  __device__ __forceinline__ S mulp(S a, S b) const {
    static_assert(SC, "needs |2^32 mod p| <= 2^22");
    return fp_redc1(fp_fold(mul64(a, b), k), k);
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

// Every complex vector is held with its time component multiplied by i (the
// loaders apply it; it is exact: the two parts swap and one changes sign).
// For x~ = (i x^0, x^1, ..., x^{d-1}) the plain sum of component products is
// sum_mu x~_mu y~_mu = -x^0 y^0 + sum_k x^k y^k = -(x.y), and the map is
// linear, so currents built from such vectors carry it too.  Dot products
// are then plain sums and "priming" the time component is the identity: no
// multiplication by a time sign in any dot product.  Root currents written
// to memory are mapped back (component 0 times -i).
template <int DL, int L>
struct C128Field {
  static constexpr int kDL = DL, kL = L;
  using E = cplx;
  using S = cplx;
  using A = cplx;
  static constexpr bool exact = false;

  __device__ C128Field(int) {}

  __device__ __forceinline__ E prime0(E x) const { return x; }
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
  template <int UX = 2, bool LAZY = false>
  __device__ __forceinline__ S ndot(const E* xp, const E* y) const {
    cplx t = cmul(xp[0], y[0]);
#pragma unroll
    for (int c = 1; c < DL; ++c) t = cmad(xp[c], y[c], t);
    return finish_dot(t);
  }
  // z + sum of x_c y_c over the point's lanes, for a z whose L-th part each
  // lane holds (z / L, exact for L a power of two): the lanes start their
  // partial sums from it, so no addition follows the group sum
  __device__ __forceinline__ S ndot_from(const E* xp, const E* y, cplx zpart) const {
    cplx t = cmad(xp[0], y[0], zpart);
#pragma unroll
    for (int c = 1; c < DL; ++c) t = cmad(xp[c], y[c], t);
    return finish_dot(t);
  }
  template <bool LAZY = false>
  __device__ __forceinline__ S ndot_u(const E* x, const E* y) const {
    cplx t = cmul(x[0], y[0]);
#pragma unroll
    for (int c = 1; c < DL; ++c) t = cmad(x[c], y[c], t);
    return finish_dot(t);
  }
  template <int UX = 2, int UZ = 2, bool LAZY = false>
  __device__ __forceinline__ S ndot_sub(const E* xp, const E* y, S z) const {
    return csub(ndot(xp, y), z);
  }
  __device__ __forceinline__ void axpy(A* K, S c, const E* v) const {
#pragma unroll
    for (int i = 0; i < DL; ++i) K[i] = cmad(c, v[i], K[i]);
  }
  __device__ __forceinline__ void fold(A*) const {}
  static constexpr bool kSC = false;
  static constexpr int kPLazy = 0, kPLazyDiff = 0, kPBal = 0, kPBalDiff = 0;
  template <int UP>
  __device__ __forceinline__ void kaxpy(A* K, int&, S c, const E* v) const { axpy(K, c, v); }
  __device__ __forceinline__ void fixed_fold(A*) const {}
  __device__ __forceinline__ E finish(A K) const { return K; }
  __device__ __forceinline__ E mul(E x, S c) const { return cmul(x, c); }
  __device__ __forceinline__ S smul(S a, S b) const { return cmul(a, b); }
};

}  // namespace bg
