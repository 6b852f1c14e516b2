// Berends-Giele recursion for large n (paper Sec. 2.2) with a group of G work
// items per phase-space point and the point's current table shared in LDS.
//
// One lane per point (bg_generic.h) needs the whole table per lane, so only a
// handful of points fit a CU at n >= 9.  Here the G items of a group split the
// work of one point instead.  Ranges of one length m depend only on shorter
// ranges, so the recursion advances length by length.  Within a length, a
// work item is (range S = [i..j], the pair of cuts c and i + j - 1 - c) for
// i <= c < j (one cut when the two coincide):
//
//   the three-gluon split A = [i..c] | B = [c+1..j] of each cut,
//   every four-gluon split [i..c] | [c+1..t] | [t+1..j] (c < t < j) of each,
//   the two adjacent-pair terms of the four-gluon vertex that pair J_A or
//   J_B with the stored -D/2 of the other part (see bg_kernel.h),
//
// summing its contribution to K'(S) over the full d components in its lanes.
// The pair evens out the four-gluon splits: every item of a length does the
// same work (two cuts, m - 2 splits), so the lanes of a wave run the same
// code.  A range's ceil((m - 1) / 2) items sit in a block of `per` item slots
// (the next power of two), a round holds G / per ranges, and after each round
// the items of a range add their sums with a butterfly across their lanes (a
// fixed order that gives every lane the same value); the first item then
// finishes S: J(S) = 2 K'(S) / P_S^2 into the LDS table, or at the root
// M = 2 eps_n . K'.  One wave barrier per length; the result does not depend
// on timing.
//
// Sub-range momenta.  F_p: exact prefix sums Q_l, P_S = Q_{j+1} - Q_i.
// Complex: prefix sums of the primed momenta held as unevaluated sums hi + lo
// (an error-free two-sum at every leg), and P_S = (hi_{j+1} - hi_i) +
// (lo_{j+1} - lo_i): the difference of the high parts rounds once, relative
// to P_S itself, so P_S is as accurate as a direct sum of its legs, where a
// difference of plain prefix sums loses the digits by which the partial sums
// exceed P_S.
//
// Same identities as the register kernel; the sum over splits is taken in the
// schedule's order, which changes only the rounding of the complex path.
// F_p propagator inverses: each item inverts its share of the denominators
// with one batched inversion and one Fermat power.
//
// Component split.  With Fld = C128Field<DL, LC> or FpField<DL, LC>, LC > 1,
// each work item belongs to LC adjacent lanes that hold DL = DMAX / LC
// components each and sum dot products over DPP: LC times the lanes per point
// for the same LDS footprint, which is what limits how many points a CU holds
// at large n.
//
// LDS access.  A lane reads whole table rows, with 16-byte reads (complex
// elements are 16 bytes; F_p rows when they start on 16-byte boundaries).
// The lanes of a wave read rows of unrelated ranges at once, so a row stride
// that is a multiple of 64 bytes (complex d = 4 or 8) sends most of them to
// the same banks; the padded layouts round a row up to an odd number of
// 16-byte units.
#pragma once

#include <type_traits>

#include "bg.h"
#include "bg_generic.h"

namespace bg {

template <class Fld, int DMAX, int G, bool PAD>
struct WideLayout {
  using E = typename Fld::E;
  using S = typename Fld::S;
  static constexpr bool kFp = Fld::exact;
  // row stride (elements) of the vector tables.  PAD makes a row an odd
  // number of 16-byte units (complex: an odd element count; F_p: 4 or 12
  // elements), so that rows start on every 16-byte bank group in turn and
  // F_p rows can be read with 16-byte loads
  static constexpr int kS = !PAD ? DMAX : (kFp ? 4 * (((DMAX + 3) / 4) | 1) : (DMAX | 1));
  static_assert(Fld::kDL * Fld::kL >= DMAX && Fld::kDL * Fld::kL <= kS, "the lanes of an item cover a row");
  // F_p rows, and each lane's part of a row, on 16-byte boundaries (the
  // table bases are 16-byte aligned)
  static constexpr bool kVec4 = kFp && kS % 4 == 0 && Fld::kDL % 4 == 0;
  struct Off {
    unsigned J, mom, epsn, nDh, nc, inv, flags, total;
  };
  __host__ __device__ static int ncur(int N) { return N * (N + 1) / 2 - 1; }
  __host__ __device__ static unsigned up16(size_t x) { return (unsigned)((x + 15) / 16 * 16); }
  // per-point LDS offsets (bytes): current table [range][component], prefix
  // sums Q_0..Q_N [leg][component] (complex: the high parts, then the low
  // parts), eps_n, scalars by range index, flags.  A vector is contiguous, so
  // a lane reads it with wide LDS loads.
  __host__ __device__ static Off offsets(int N) {
    Off o{};
    unsigned x = 0;
    o.J = x;      x += up16((size_t)ncur(N) * kS * sizeof(E));
    o.mom = x;    x += up16((size_t)(kFp ? 1 : 2) * (N + 1) * kS * sizeof(E));
    o.epsn = x;   x += up16((size_t)DMAX * sizeof(E));
    o.nDh = x;    x += up16((size_t)ncur(N) * sizeof(S));
    o.nc = x;     x += kFp ? up16((size_t)ncur(N) * sizeof(S)) : 0u;
    o.inv = x;    x += kFp ? up16((size_t)ncur(N) * sizeof(S)) : 0u;
    o.flags = x;  x += 16;
    o.total = x;
    return o;
  }
};

// The G items of a group lie in one wavefront (G LC divides 64), so a group
// needs no workgroup barrier: waiting for this wave's LDS operations and
// keeping the compiler from moving LDS accesses across the point is enough.
__device__ __forceinline__ void group_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// the value of lane (this lane XOR ST): ds_swizzle in bit mode within 32
// lanes, ds_bpermute across the halves of the wave
template <int ST>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  static_assert(ST >= 1 && ST <= 32 && (ST & (ST - 1)) == 0, "a lane distance that is a power of two");
  if constexpr (ST < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (ST << 10));
  else return (uint32_t)__builtin_amdgcn_ds_bpermute((int)((__lane_id() ^ ST) << 2), (int)v);
}
template <int ST>
__device__ __forceinline__ int64_t lane_xor(int64_t v) {
  u32x2 p = __builtin_bit_cast(u32x2, v);
  p.x = lane_xor<ST>(p.x);
  p.y = lane_xor<ST>(p.y);
  return __builtin_bit_cast(int64_t, p);
}
template <int ST>
__device__ __forceinline__ double lane_xor(double v) {
  return __builtin_bit_cast(double, lane_xor<ST>(__builtin_bit_cast(int64_t, v)));
}
template <int ST>
__device__ __forceinline__ cplx lane_xor(cplx v) {
  return cplx{lane_xor<ST>(v.re), lane_xor<ST>(v.im)};
}

template <class Fld, int DMAX, int G, bool PAD>
struct WideRecursion {
  using E = typename Fld::E;
  using S = typename Fld::S;
  using A = typename Fld::A;
  using Lay = WideLayout<Fld, DMAX, G, PAD>;
  static constexpr int kS = Lay::kS;
  static constexpr int DL = Fld::kDL;   // components per lane
  static constexpr int LC = Fld::kL;    // lanes per work item
  using Rec = Recursion<Fld, 2, DL, LC>;  // scalar helpers
  static constexpr bool kFp = Fld::exact;
  // per-item sum of the -(J_A . J_B) of its cuts: F_p an int64 sum of
  // products with 1/2, complex the plain sum
  using NDS = std::conditional_t<kFp, int64_t, S>;

  E* Jt;
  E* Mt;
  E* Ml;
  E* En;
  S* nDht;
  S* nct;
  S* invt;
  unsigned* flags;
  int N, g, s, ln, co;  // item slot, component part, lane in the point, first component

  __device__ WideRecursion(char* base, int N_, int ln_)
      : N(N_), g(ln_ / LC), s(ln_ % LC), ln(ln_), co((ln_ % LC) * DL) {
    const auto o = Lay::offsets(N);
    Jt = reinterpret_cast<E*>(base + o.J);
    Mt = reinterpret_cast<E*>(base + o.mom);
    Ml = Mt + (N + 1) * kS;  // complex: low parts of the prefix sums
    En = reinterpret_cast<E*>(base + o.epsn);
    nDht = reinterpret_cast<S*>(base + o.nDh);
    nct = reinterpret_cast<S*>(base + o.nc);
    invt = reinterpret_cast<S*>(base + o.inv);
    flags = reinterpret_cast<unsigned*>(base + o.flags);
  }

  __device__ __forceinline__ int rid(int i, int j) const { return range_idx(N, i, j); }
  __device__ __forceinline__ E& Jat(int r, int c) const { return Jt[r * kS + c]; }
  __device__ __forceinline__ E& Mat(int l, int c) const { return Mt[l * kS + c]; }
  __device__ __forceinline__ E& Mlo(int l, int c) const { return Ml[l * kS + c]; }
  // one table row into registers with 16-byte LDS reads where the layout
  // allows (complex elements are 16 bytes; F_p rows of a padded layout start
  // on 16-byte boundaries)
  __device__ __forceinline__ static void load_row(const E* row, E (&x)[DL]) {
    if constexpr (!kFp) {
      const double2* p = reinterpret_cast<const double2*>(row);
#pragma unroll
      for (int c = 0; c < DL; ++c) {
        const double2 v = p[c];
        x[c] = cplx{v.x, v.y};
      }
    } else if constexpr (Lay::kVec4) {
      const int4* p4 = reinterpret_cast<const int4*>(row);
#pragma unroll
      for (int q = 0; q < DL / 4; ++q) {
        const int4 v = p4[q];
        x[4 * q] = v.x;
        x[4 * q + 1] = v.y;
        x[4 * q + 2] = v.z;
        x[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int c = 0; c < DL; ++c) x[c] = row[c];
    }
  }
  // this lane's components of a row
  __device__ __forceinline__ void loadJ(int r, E (&x)[DL]) const { load_row(Jt + r * kS + co, x); }
  __device__ __forceinline__ void loadM(int l, E (&x)[DL]) const { load_row(Mt + l * kS + co, x); }
  // complex: prefix sum Q_l as its high and low parts
  __device__ __forceinline__ void loadQ(int l, E (&h)[DL], E (&lo)[DL]) const {
    load_row(Mt + l * kS + co, h);
    load_row(Ml + l * kS + co, lo);
  }
  // complex: primed P of the legs between two prefix sums, (hb - ha) + (lb - la)
  __device__ __forceinline__ static void dd_diff(const E (&ha)[DL], const E (&la)[DL], const E (&hb)[DL],
                                                 const E (&lb)[DL], E (&P)[DL]) {
#pragma unroll
    for (int c = 0; c < DL; ++c) P[c] = cadd(csub(hb[c], ha[c]), csub(lb[c], la[c]));
  }
  // F_p: primed P_S, reduced, from prefix sums
  __device__ __forceinline__ void primedP(const Fld& F, int i, int j, E (&P)[DL]) const {
    E a[DL], b[DL];
    loadM(j + 1, a);
    loadM(i, b);
#pragma unroll
    for (int c = 0; c < DL; ++c) P[c] = F.esub(a[c], b[c]);
    P[0] = F.prime0(P[0]);
  }
  // F_p: primed P_S as unreduced differences Q_{j+1} - Q_i (|slot| <= 2h)
  __device__ __forceinline__ void lazyP(const Fld& F, int i, int j, E (&P)[DL]) const {
    E a[DL], b[DL];
    loadM(j + 1, a);
    loadM(i, b);
#pragma unroll
    for (int c = 0; c < DL; ++c) P[c] = a[c] - b[c];
    P[0] = F.prime0(P[0]);
  }

  // F_p: lazyP, and Q_i + Q_{j+1} unreduced (|slot| <= 2h) from the same rows
  __device__ __forceinline__ void lazyPQ(const Fld& F, int i, int j, E (&P)[DL], E (&QQ)[DL]) const {
    E a[DL], b[DL];
    loadM(j + 1, a);
    loadM(i, b);
#pragma unroll
    for (int c = 0; c < DL; ++c) {
      P[c] = a[c] - b[c];
      QQ[c] = a[c] + b[c];
    }
    P[0] = F.prime0(P[0]);
  }

  // ---- loads: eps into the table, momenta, eps_n; prefix sums -------------
  __device__ void load(const Fld& F, const LaunchArgs& a, int64_t q, uint32_t& bad) {
    // every global load of the point first (a fixed count per lane, the
    // ones past the last row repeat row 0), then the LDS stores
    constexpr int kLegs = BG_MAX_N - 1;                        // N <= 13
    constexpr int kRowsMax = (2 * kLegs + 1) * DMAX;           // eps_0..eps_N, k_0..k_{N-1}
    constexpr int kIt = (kRowsMax + G * LC - 1) / (G * LC);
    const int rows = (2 * N + 1) * DMAX;
    E v[kIt];
#pragma unroll
    for (int t = 0; t < kIt; ++t) {
      const int r = ln + t * G * LC;
      const int rr = r < rows ? r : 0;
      const int which = rr / DMAX, c = rr % DMAX;
      const bool eps = which <= N;
      v[t] = Loader<Fld>::template get<MetricRT>(a, eps ? a.pols : a.momenta, eps ? which : which - N - 1, c, q,
                                                 bad);
    }
#pragma unroll
    for (int t = 0; t < kIt; ++t) {
      const int r = ln + t * G * LC;
      if (r < rows) {
        const int which = r / DMAX, c = r % DMAX;
        // eps_l into the table, eps_n aside, raw k_l (complex: primed,
        // which is the identity) into the prefix-sum rows, summed below
        E* dst = which < N ? &Jat(rid(which, which), c) : (which == N ? &En[c] : &Mat(which - N, c));
        *dst = v[t];
      }
    }
    if (ln == 0) *flags = 0u;
    if (ln < N) nDht[rid(ln, ln)] = S{};  // a single leg has no two-way split
    group_sync();
    if (ln < DMAX) {  // prefix sums, one component per lane: all legs read first
      E k[kLegs];
#pragma unroll
      for (int l = 0; l < kLegs; ++l) k[l] = l < N ? Mat(l + 1, ln) : E{};
      if constexpr (kFp) {
        E acc{};
        Mat(0, ln) = acc;
#pragma unroll
        for (int l = 0; l < kLegs; ++l) {
          if (l < N) {
            acc = F.eadd(acc, k[l]);
            Mat(l + 1, ln) = acc;
          }
        }
      } else {
        // hi + lo = Q_l exactly up to the rounding of lo: hi takes the
        // two-sum with each leg, lo collects the rounding errors
        double hr = 0.0, hm = 0.0, lr = 0.0, lm = 0.0;
        Mat(0, ln) = cplx{0.0, 0.0};
        Mlo(0, ln) = cplx{0.0, 0.0};
#pragma unroll
        for (int l = 0; l < kLegs; ++l) {
          if (l < N) {
            const double sr = hr + k[l].re, br = sr - hr;
            lr += (hr - (sr - br)) + (k[l].re - br);
            hr = sr;
            const double sm = hm + k[l].im, bm = sm - hm;
            lm += (hm - (sm - bm)) + (k[l].im - bm);
            hm = sm;
            Mat(l + 1, ln) = cplx{hr, hm};
            Mlo(l + 1, ln) = cplx{lr, lm};
          }
        }
      }
    }
    group_sync();
    if constexpr (kFp) {
      for (int l = g; l < N; l += G) {  // nc(l) = P_l . eps_l
        E Pp[DL], e[DL];
        lazyP(F, l, l, Pp);
        loadJ(rid(l, l), e);
        nct[rid(l, l)] = F.template ndot<4>(Pp, e);
      }
    }
  }

  // ---- F_p: -P_S^2 for every 2 <= |S| <= N-1, inverted per lane ---------
  __device__ void inverses(const Fld& F, bool& singular) {
    if constexpr (kFp) {
      const int np = N * (N - 1) / 2 - 1;  // ranges of length 2..N-1 have indices N .. N+np-1
      int32_t acc = F.k.one;
      bool any = false;
      for (int r = g; r < np; r += G) {  // forward: y into invt, prefix products into nDht
        const int id = N + r;
        int len = 2, base = 0;
        while (r >= base + (N - len + 1)) { base += N - len + 1; ++len; }
        const int i = r - base;
        E Pp[DL], Pu[DL];
        primedP(F, i, i + len - 1, Pp);
#pragma unroll
        for (int c = 0; c < DL; ++c) Pu[c] = Pp[c];
        Pu[0] = F.prime0(Pp[0]);
        int32_t y = F.ndot(Pp, Pu);
        if (y == 0) { singular = true; y = F.k.one; }
        acc = any ? fp_mul(acc, y, F.k) : y;
        any = true;
        invt[id] = y;
        nDht[id] = acc;
      }
      if (any) {
        int32_t t = fp_pow(acc, (uint32_t)(F.k.p - 2), F.k);
        // 1/y = -1/P^2 -> 2/P^2, with the extra 2^-32 that finish_mul32 expects
        t = fp_mul(t, -F.k.two32, F.k);
        int last = g;
        while (last + G < np) last += G;
        for (int r = last; r >= g; r -= G) {
          const int id = N + r;
          const int32_t y = invt[id];
          invt[id] = r > g ? fp_mul(t, nDht[id - G], F.k) : t;
          t = fp_mul(t, y, F.k);
        }
      }
    }
  }

  // ---- one three-gluon cut: contributions of cut c to K'(S), S = [i..j] ---
  // the split [i..c] | [c+1..j] and the adjacent-pair terms of the four-gluon
  // vertex that involve this cut.  F_p: Pp holds P_S as unreduced
  // differences, nDs accumulates -(J_A.J_B) / 2 as an int64 sum of products;
  // complex: PA, PB are the primed P_A, P_B (Pp unused), nDs sums -(J_A.J_B).
  __device__ void cut3(const Fld& F, int i, int j, int c, const E (&Pp)[DL], const E (&PA)[DL],
                       const E (&PB)[DL], A (&K)[DL], NDS& nDs) const {
    E JA[DL], JB[DL];
    const int ra = rid(i, c), rb = rid(c + 1, j);
    loadJ(ra, JA);
    loadJ(rb, JB);
    const S nDm = F.ndot_u(JA, JB);  // -(J_A . J_B)
    if constexpr (kFp) {
      // the adjacent-pair terms -Dh(A) J_B and -Dh(B) J_A join the scalars
      // of the J_B and J_A axpys: -Dh (balanced, zero for a single leg),
      // lifted by R, enters each dot product's accumulator before its REDC
      E Qt[DL];
      loadM(c + 1, Qt);
      const S nc2 = F.template ndot_sub2<4, 2, false, 2>(Pp, JA, nct[ra], nDht[ra]);            // -(P_B.J_A) + Dh(A)
      const S nc3 = F.template ndot_sub2<4, 2, false, 2>(Pp, JB, nct[rb], F.sneg(nDht[rb]));   // -(P_A.J_B) - Dh(B)
      F.axpy(K, F.sneg(nDm), Qt);
      F.axpy(K, F.sneg(nc2), JB);
      F.axpy(K, nc3, JA);
      nDs = fp_fold(mad64(nDm, F.k.inv2, nDs), F.k);
    } else {
      // the adjacent-pair terms: the lanes of the item start their partial
      // dot products from their share of -Dh (the table holds -Dh / LC, zero
      // for a single leg)
      E v[DL];
      const S n2 = F.ndot_from(PB, JA, cneg(nDht[ra]));  // -(P_B.J_A) + Dh(A), negated below
      const S n3 = F.ndot_from(PA, JB, nDht[rb]);        // -(P_A.J_B) - Dh(B)
#pragma unroll
      for (int x = 0; x < DL; ++x) v[x] = F.esub(PA[x], PB[x]);
      v[0] = F.prime0(v[0]);  // P_A - P_B
      F.axpy(K, cplx{-0.5 * nDm.re, -0.5 * nDm.im}, v);
      F.axpy(K, F.sneg(n2), JB);
      F.axpy(K, n3, JA);
      nDs = cadd(nDs, nDm);
    }
    // F_p: K is folded by the caller, once after the item's cuts
  }

  // ---- four-gluon splits [i..c] | [c+1..t] | [t+1..j] of a pair of cuts --
  // j - c1 - 1 splits of cut c1, then j - c2 - 1 of cut c2 (none when
  // c2 == c1), in one loop: the two cuts of a pair have m - 2 splits together,
  // so every lane of a round runs the same number of iterations.  Range
  // indices advance incrementally: with e = (right end - left end) of a range,
  // extending [c+1..t] to [c+1..t+1] adds N - e, and shrinking [t+1..j] to
  // [t+2..j] adds e - N (from the index formula of range_idx).
  __device__ void cut4(const Fld& F, int i, int j, int c1, int c2, A (&K)[DL]) const {
    E JA[DL];
    loadJ(rid(i, c1), JA);
    const int n1 = j - c1 - 1;
    const int nt = n1 + (c2 != c1 ? j - c2 - 1 : 0);
    int rm = rid(c1 + 1, c1 + 1), lm = 0;
    int rc = rid(c1 + 2, j), lc = j - c1 - 2;
    int cnt = 0;
#pragma unroll 2
    for (int q = 0; q < nt; ++q) {
      if (q == n1) {  // on to cut c2 (only reached when it has splits)
        loadJ(rid(i, c2), JA);
        rm = rid(c2 + 1, c2 + 1);
        lm = 0;
        rc = rid(c2 + 2, j);
        lc = j - c2 - 2;
      }
      E JM[DL], JC[DL];
      loadJ(rm, JM);
      loadJ(rc, JC);
      const S ne = F.ndot_u(JA, JC);
      F.axpy(K, F.sneg(ne), JM);
      if (++cnt == 5) { F.fold(K); cnt = 0; }
      rm += N - lm;
      ++lm;
      rc += lc - N;
      --lc;
    }
    F.fold(K);
  }

  // the sums of the per items of each range (lanes LC apart), added in a
  // butterfly: every lane of the range ends with the same total
  template <int ST>
  __device__ __forceinline__ void xor_step(const Fld& F, A (&K)[DL], NDS& nDs) const {
#pragma unroll
    for (int c = 0; c < DL; ++c) K[c] = add_acc(F, K[c], lane_xor<ST>(K[c]));
    if constexpr (kFp) nDs = fp_fold(nDs + lane_xor<ST>(nDs), F.k);
    else nDs = cadd(nDs, lane_xor<ST>(nDs));
  }
  __device__ __forceinline__ void range_sum(const Fld& F, A (&K)[DL], NDS& nDs, int per) const {
    // per is the same in every lane of the wave (all its points have this N)
    if constexpr (LC <= 32) if (per > 1) xor_step<LC>(F, K, nDs);
    if constexpr (LC * 2 <= 32) if (per > 2) xor_step<LC * 2>(F, K, nDs);
    if constexpr (LC * 4 <= 32) if (per > 4) xor_step<LC * 4>(F, K, nDs);
    if constexpr (LC * 8 <= 32) if (per > 8) xor_step<LC * 8>(F, K, nDs);
    if constexpr (LC * 16 <= 32) if (per > 16) xor_step<LC * 16>(F, K, nDs);
    if constexpr (LC * 32 <= 32) if (per > 32) xor_step<LC * 32>(F, K, nDs);
  }

  __device__ void run(const Fld& F, const LaunchArgs& a, int64_t q, S& result, E (&kroot)[DL]) {
    uint32_t bad = 0;
    bool singular = false;
    load(F, a, q, bad);
    inverses(F, singular);
    group_sync();

    for (int m = 2; m <= N; ++m) {
      const int nr = N - m + 1;        // ranges of length m: i = 0 .. nr-1
      const int pairs = m / 2;         // items per range: cuts c and i + j - 1 - c
      int lg = 0;                      // per = 2^lg item slots per range
      while ((1 << lg) < pairs) ++lg;
      const int per = 1 << lg, rpr = G >> lg;  // ranges per round
      const int rl = g >> lg, u = g & (per - 1);
      for (int r0 = 0; r0 < nr; r0 += rpr) {  // rounds of G / per ranges
        const int r = r0 + rl;
        const bool act = r < nr && u < pairs;
        A K[DL];
#pragma unroll
        for (int c = 0; c < DL; ++c) K[c] = F.azero();
        NDS nDs{};
        // what the range's finish needs and K does not (P_S, the propagator
        // inverse, F_p: Q_i + Q_{j+1}): formed before the cuts, so that its
        // loads and the division overlap their work
        E Pp[DL], QQ[DL];
        S inv2{};
        if constexpr (kFp) {
          // every slot of the range finishes some of its components
          if (r < nr) {
            lazyPQ(F, r, r + m - 1, Pp, QQ);
            if (m < N) inv2 = invt[rid(r, r + m - 1)];
          }
        }
        if (act) {
          const int i = r, j = r + m - 1;
          const int c1 = i + u, c2 = j - 1 - u;
          if constexpr (kFp) {
            cut3(F, i, j, c1, Pp, Pp, Pp, K, nDs);
            if (c2 != c1) cut3(F, i, j, c2, Pp, Pp, Pp, K, nDs);
            F.fold(K);  // two cuts' products from zero fit the accumulator
          } else {
            E Qih[DL], Qil[DL], Qjh[DL], Qjl[DL], Qch[DL], Qcl[DL], PA[DL], PB[DL];
            loadQ(i, Qih, Qil);
            loadQ(j + 1, Qjh, Qjl);
            dd_diff(Qih, Qil, Qjh, Qjl, Pp);
            if (m < N) {  // the root has no propagator
              E Pu[DL];
#pragma unroll
              for (int c = 0; c < DL; ++c) Pu[c] = Pp[c];
              Pu[0] = F.prime0(Pp[0]);
              inv2 = Rec::c_inverse_times(F.ndot(Pp, Pu), -2.0, singular);
            }
            loadQ(c1 + 1, Qch, Qcl);
            dd_diff(Qih, Qil, Qch, Qcl, PA);
            dd_diff(Qch, Qcl, Qjh, Qjl, PB);
            cut3(F, i, j, c1, Pp, PA, PB, K, nDs);
            if (c2 != c1) {
              loadQ(c2 + 1, Qch, Qcl);
              dd_diff(Qih, Qil, Qch, Qcl, PA);
              dd_diff(Qch, Qcl, Qjh, Qjl, PB);
              cut3(F, i, j, c2, Pp, PA, PB, K, nDs);
            }
          }
          cut4(F, i, j, c1, c2, K);
        }
        if constexpr (kFp) {
          if (m < N) {
            scalar_sum<LC>(F, nDs, lg);
            if (r < nr) rs_finish<LC, DL>(F, K, QQ, Pp, lg, 0, 1, nDs, inv2, rid(r, r + m - 1), u == 0, lg);
            continue;
          }
        }
        range_sum(F, K, nDs, per);
        if (act && u == 0) {  // the range's first item finishes it
          const int id = rid(r, r + m - 1);
          S nDhS;
          if constexpr (kFp) {
            nDhS = fp_redc2(fp_fold(nDs, F.k), F.k);  // the cuts' sums already carry the factor 1/2
            // -Dh(S) (Q_i + Q_{j+1})
            F.axpy(K, nDhS, QQ);
            F.fold(K);
          } else {
            constexpr double kPart = 0.5 / Fld::kL;  // -Dh(S) / LC, the lanes' share
            nDhS = cplx{kPart * nDs.re, kPart * nDs.im};
          }
          if (m < N) {
            nDht[id] = nDhS;
            E Jn[DL];
#pragma unroll
            for (int c = 0; c < DL; ++c) {
              if constexpr (kFp) Jn[c] = F.finish_mul32(K[c], inv2);
              else Jn[c] = F.mul(F.finish(K[c]), inv2);
              Jat(id, co + c) = Jn[c];
            }
            if constexpr (kFp) nct[id] = F.template ndot<4>(Pp, Jn);
          } else {
            E Kf[DL], en[DL];
#pragma unroll
            for (int c = 0; c < DL; ++c) {
              Kf[c] = F.finish(K[c]);
              en[c] = En[co + c];
            }
            result = F.ndot_u(en, Kf);
#pragma unroll
            for (int c = 0; c < DL; ++c) kroot[c] = Kf[c];
          }
        }
      }
      group_sync();
    }
    // per-point flags: bit 0 bad residue (F_p), bit 1 singular
    unsigned fl = singular ? 2u : 0u;
    if constexpr (kFp) fl |= bad >= (uint32_t)F.k.p ? 1u : 0u;
    if (fl) atomicOr(flags, fl);
    group_sync();
  }

  // ---- F_p, ranges shorter than the point: reduce-scatter, then a finish
  // spread over the range's slots.  After the cuts every slot of a range
  // holds partial sums of all DL components of K.  A step at lane distance
  // ST halves what a slot holds: of each pair of components it keeps the one
  // its bit selects, adding the partner's partial of it, and sends the other
  // one.  After the steps a slot holds the complete sums of DN components of
  // the lane's part (component cb + q cs); steps left when DN is odd add
  // whole values.  Each slot then finishes its components; P_S . J_S is
  // summed over the slots that hold different components.
  template <int ST>
  __device__ __forceinline__ void scalar_sum(const Fld& F, int64_t& x, int lg) const {
    if constexpr (ST <= 32) {
      if (lg > 0) {
        x = fp_fold(x + lane_xor<ST>(x), F.k);
        scalar_sum<ST * 2>(F, x, lg - 1);
      }
    }
  }
  template <int ST, int DN>
  __device__ __forceinline__ void rest_sum(const Fld& F, A (&V)[DN], int lg) const {
    if constexpr (ST <= 32) {
      if (lg > 0) {
#pragma unroll
        for (int q = 0; q < DN; ++q) V[q] = add_acc(F, V[q], lane_xor<ST>(V[q]));
        rest_sum<ST * 2, DN>(F, V, lg - 1);
      }
    }
  }
  template <int ST, int DN>
  __device__ __forceinline__ void rs_finish(const Fld& F, const A (&V)[DN], const E (&Qv)[DN], const E (&Pv)[DN], int lg, int cb,
                            int cs, int64_t nDs, S inv2, int id, bool first, int lgall) const {
    if constexpr (DN % 2 == 0 && ST <= 32) {
      if (lg > 0) {
        const bool b = (ln & ST) != 0;
        A W[DN / 2];
        E Qh[DN / 2], Ph[DN / 2];
#pragma unroll
        for (int p = 0; p < DN / 2; ++p) {
          const A send = b ? V[2 * p] : V[2 * p + 1];
          const A keep = b ? V[2 * p + 1] : V[2 * p];
          W[p] = add_acc(F, keep, lane_xor<ST>(send));
          // opaque copies: a select between two elements of one array would
          // otherwise become an indexed load, with the array in scratch memory
          E q0 = Qv[2 * p], q1 = Qv[2 * p + 1], p0 = Pv[2 * p], p1 = Pv[2 * p + 1];
          asm volatile("" : "+v"(q0), "+v"(q1), "+v"(p0), "+v"(p1));
          Qh[p] = b ? q1 : q0;
          Ph[p] = b ? p1 : p0;
        }
        rs_finish<ST * 2, DN / 2>(F, W, Qh, Ph, lg - 1, b ? cb + cs : cb, cs * 2, nDs, inv2, id, first, lgall);
        return;
      }
    }
    // after the lg steps left here, the 2^lg slots that differ only in the
    // higher bits hold the same components
    A K[DN];
#pragma unroll
    for (int q = 0; q < DN; ++q) K[q] = V[q];
    rest_sum<ST, DN>(F, K, lg);
    const S nDhS = fp_redc2(fp_fold(nDs, F.k), F.k);  // the cuts' sums already carry the factor 1/2
    A t = 0;
    int uu = 0;
#pragma unroll
    for (int q = 0; q < DN; ++q) {
      // -Dh(S) (Q_i + Q_{j+1}), then J = K' 2/P_S^2
      const E Jn = F.finish_mul32(fp_fold(mad64(nDhS, Qv[q], K[q]), F.k), inv2);
      Jat(id, co + cb + q * cs) = Jn;
      // P_S . J_S over this slot's components (an unreduced difference times
      // a balanced value: the dot products' UX = 4 class)
      if (uu + Fld::ux_units(4) > Fld::kMaxU) {
        t = fp_fold(t, F.k);
        uu = Fld::kFoldU;
      }
      t = mad64(Pv[q], Jn, t);
      uu += Fld::ux_units(4);
    }
    t = fp_fold(t, F.k);
    scalar_sum<LC>(F, t, lgall - lg);  // over the slots whose components differ
    const S nc = F.template finish_dot<false>(t, Fld::kFoldU);
    if (first) {
      nct[id] = nc;
      nDht[id] = nDhS;
    }
  }

  // K + partial (F_p: both below 2^61 + 2^32 after their folds, refolded)
  __device__ __forceinline__ static A add_acc(const Fld& F, A x, A y) {
    if constexpr (kFp) return fp_fold(x + y, F.k);
    else return cadd(x, y);
  }
};

// One point of a lane-group launch: the G LC lanes of point slot pb of the
// block (lane t of the point) compute point q0 of the launch described by a,
// with the point's tables at lds + pb * WideLayout::offsets(N).total.
template <class Fld, int DMAX, int G, bool PAD>
__device__ __forceinline__ void wide_point(const LaunchArgs& a, int N, char* lds, int pb, int t, int64_t q0) {
  using Lay = WideLayout<Fld, DMAX, G, PAD>;
  using WR = WideRecursion<Fld, DMAX, G, PAD>;
  const bool valid = q0 < a.npts;
  const int64_t q = valid ? q0 : a.npts - 1;  // tail groups recompute the last point
  WR W(lds + (size_t)pb * Lay::offsets(N).total, N, t);
  typename Fld::S res;
  typename Fld::E kroot[WR::DL];
  if constexpr (Fld::exact) {
    Fld F(a.fp, W.s);
    W.run(F, a, q, res, kroot);
    // the lanes of item slot 0 hold the root, DL components each
    if (valid && W.g == 0) {
      const unsigned fl = *W.flags;
      const uint8_t st = (fl & 1u) ? PT_BADRESIDUE : ((fl & 2u) ? PT_SINGULAR : PT_OK);
      if (a.cur) {
        // root current K = 2 K', kroot scaled by R^-3: one product with R^3
#pragma unroll
        for (int c = 0; c < WR::DL; ++c) {
          const int mu = W.co + c;
          if (mu < a.d) {
            uint32_t v = 0xFFFFFFFFu;
            if (st == PT_OK) {
              const int32_t m = fp_mul(kroot[c], a.fp.r3, a.fp);
              v = fp_to_canonical(fp_add(m, m, a.fp), a.fp);
            }
            static_cast<uint32_t*>(a.cur)[(int64_t)mu * a.ld + q] = v;
          }
        }
      } else if (W.s == 0) {
        uint32_t outv = 0xFFFFFFFFu;
        if (st == PT_OK) {
          int32_t m = fp_mul(res, a.fp.r4, a.fp);
          m = fp_sub(0, fp_add(m, m, a.fp), a.fp);
          outv = fp_to_canonical(m, a.fp);
        }
        static_cast<uint32_t*>(a.out)[q] = outv;
      }
      if (a.status && W.s == 0) a.status[q] = st;
    }
  } else {
    Fld F(W.s);
    W.run(F, a, q, res, kroot);
    // the lanes of item slot 0 hold the root current, DL components each
    if (valid && W.g == 0) {
      const bool sing = (*W.flags & 2u) != 0;
      if (a.cur) {
#pragma unroll
        for (int c = 0; c < WR::DL; ++c) {
          const int mu = W.co + c;
          if (mu < a.d) {
            double2 o;
            // component 0 back from its factor i: K^0 = -i (i K^0)
            const cplx k = mu == 0 ? cplx{kroot[c].im, -kroot[c].re} : kroot[c];
            o.x = sing ? __builtin_nan("") : 2.0 * k.re;
            o.y = sing ? __builtin_nan("") : 2.0 * k.im;
            static_cast<double2*>(a.cur)[(int64_t)mu * a.ld + q] = o;
          }
        }
      } else if (W.s == 0) {
        double2 o;
        if (sing) {
          o.x = __builtin_nan("");
          o.y = __builtin_nan("");
        } else {
          o.x = -2.0 * res.re;
          o.y = -2.0 * res.im;
        }
        static_cast<double2*>(a.out)[q] = o;
      }
      if (a.status && W.s == 0) a.status[q] = sing ? PT_SINGULAR : PT_OK;
    }
  }
}

// G items per point, each on LC = Fld::kL adjacent lanes (G LC divides 64),
// blockDim.x / (G LC) points per block, LDS from the host (points per block x
// WideLayout::offsets(N).total bytes).
template <class Fld, int DMAX, int G, bool PAD>
__global__ __launch_bounds__(256) void bg_wide_kernel(LaunchArgs a, int N) {
  extern __shared__ __align__(16) char lds[];
  constexpr int GL = G * Fld::kL;  // lanes per point
  static_assert(G >= 16 && 64 % GL == 0, "a lane group lies in one wavefront and owns up to 13 ranges");
  const int t = (int)(threadIdx.x % GL);
  const int pb = (int)(threadIdx.x / GL);
  const int64_t q0 = (int64_t)xcd_block_index() * (blockDim.x / GL) + pb;
  wide_point<Fld, DMAX, G, PAD>(a, N, lds, pb, t, q0);
}

// ---------------------------------------------------------------------------
// persistent form over a work queue (batched launches, paper Sec. 3.2: the
// per-launch offset that a fixed set of precompiled kernels removes)
// ---------------------------------------------------------------------------
// The blocks stay resident and take tiles from the queue with one atomic
// increment each until it is empty; the group table is ordered by cost per
// point, longest first, so the expensive groups start first and the cheap
// ones fill the tail.  Every block reaches the exit: once the counter has
// passed ntiles every further increment returns a value >= ntiles.
template <class Fld, int DMAX, int G, bool PAD>
__global__ __launch_bounds__(256) void bg_wide_queue_kernel(const QueueGroup* groups, int ngroups, uint32_t ntiles,
                                                           uint32_t* next) {
  // the first 16 bytes of the block's LDS hold the current tile, the points'
  // tables follow (the host sizes the launch with kQueueLdsHeader included)
  extern __shared__ __align__(16) char lds[];
  uint32_t& tile_s = *reinterpret_cast<uint32_t*>(lds);
  constexpr int GL = G * Fld::kL;
  const int t = (int)(threadIdx.x % GL);
  const int pb = (int)(threadIdx.x / GL);
  const int P = (int)(blockDim.x / GL);
  for (;;) {
    if (threadIdx.x == 0) tile_s = atomicAdd(next, 1u);
    __syncthreads();
    // the same value in every thread of the block: kept in scalar registers,
    // so the group lookup and its arguments are scalar loads
    const uint32_t tile = __builtin_amdgcn_readfirstlane(tile_s);
    if (tile >= ntiles) return;
    int g = 0;
    while (g + 1 < ngroups && groups[g + 1].first_tile <= tile) ++g;
    const LaunchArgs a = groups[g].args;
    const int N = groups[g].N;
    const int64_t q0 = (int64_t)(tile - groups[g].first_tile) * P + pb;
    wide_point<Fld, DMAX, G, PAD>(a, N, lds + kQueueLdsHeader, pb, t, q0);
    __syncthreads();  // tile_s and the LDS tables are reused by the next tile
  }
}

}  // namespace bg
