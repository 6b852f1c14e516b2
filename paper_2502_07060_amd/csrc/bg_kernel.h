// Register-resident Berends-Giele recursion for one phase-space point per
// group of L lanes (paper Sec. 2.2).  Template over the field policy, N = n-1,
// DL = components per lane and L = lanes per point; the whole recursion is
// unrolled at compile time, so every current lives in registers.
//
// What each point computes (identities exact in any field, valid for any
// inputs; no on-shell or transversality assumption):
//
//   D(X)  = sum over splits A|B of X of J_A . J_B,  Dh = D / 2
//
// and, with K'(S) = K(S) / 2 (K the bracket of the paper's recursion once the
// factors of i are cancelled),
//
//   K'(S) = sum_{A|B} [ (1/2)(J_A.J_B)(P_A - P_B) + (P_B.J_A) J_B - (P_A.J_B) J_A ]
//         + sum_{A|B|C} (J_A.J_C) J_B
//         - sum_t Dh([i..t]) J([t+1..j]) - sum_s Dh([s+1..j]) J([i..s])
//
// The first line is the three-gluon vertex; the last two are the four-gluon
// vertex with its two adjacent-pair dot products summed into Dh.  Then
// J(S) = 2 K'(S) / P_S^2 and M = 2 eps_n . K'([1..N]).  Ranges are visited
// column by column (right end j ascending, left end i descending), so every
// range a split reads is already final.
//
// Sub-range momenta.  Over F_p every identity is exact, so with prefix sums
// Q_l = k_1 + ... + k_l, P_S = Q_{j+1} - Q_i, c(X) = P_X . J_X one has
// P_B.J_A = P_S.J_A - c(A), P_A.J_B = P_S.J_B - c(B) and
// P_A - P_B = 2 Q_{a+1} - Q_i - Q_{j+1}: no vector of momenta is formed per
// split.  Over C the momenta are summed left to right exactly as the
// definition P_{i,j} = k_i + ... + k_j reads (the column P_{i..j} for the
// current j, and P_A grown along the split loop), which keeps the rounding of
// small sub-range momenta independent of the size of the partial sums; the
// first term is taken as (J_A.J_B) P_A per split and -(1/2) D(S) P_S once.
#pragma once

#include "bg_common.h"
#include "bg_fields.h"

#ifndef BG_SPLIT_BARRIER
#define BG_SPLIT_BARRIER 1
#endif
// instruction classes the scheduler may still move across a split barrier
// (sched_barrier mask; 0: none)
#ifndef BG_SPLIT_BARRIER_MASK
#define BG_SPLIT_BARRIER_MASK 0
#endif

namespace bg {

enum { PT_OK = 0, PT_SINGULAR = 1, PT_BADRESIDUE = 2 };

struct LaunchArgs {
  const void* momenta;
  const void* pols;
  void* out;
  uint8_t* status;
  int64_t npts;
  int64_t ld;
  int d;
  FpConst fp;  // F_p only
  // metric: 0 mostly-minus; 1 alternating diag(1, -1, 1, -1, ...), mapped onto
  // the mostly-minus one on load (see Loader)
  int metric;
  int32_t ialt;  // F_p: factor of the components 2, 4, ... at load: a square root of -1 times R
                 // in the alternating metric, R (Montgomery one) in the mostly-minus one
  // root-current mode: when non-null, the kernels write K([1..n-1]) (d
  // components, [d][ld]) here instead of M to `out`
  void* cur;
};

// One group of a persistent queue launch (bg_wide_queue_kernel): its launch
// arguments, N = n - 1, and the first tile of the group in queue order (tiles
// of a fixed number of points per launch).
struct QueueGroup {
  LaunchArgs args;
  int N;
  uint32_t first_tile;
};
constexpr unsigned kQueueLdsHeader = 16;  // LDS bytes before the points' tables

// ---------------------------------------------------------------------------
// loads
// ---------------------------------------------------------------------------
// Every load is unconditional (a padded component reads row 0 and is zeroed
// afterwards), so the compiler can issue all of a point's loads back to back
// and wait once.  On F_p the largest raw residue seen is kept in `maxraw`;
// the point has a bad residue iff it ends up >= p.
//
// Alternating metric (paper Sec. 3.1, diag(1, -1, 1, -1, ...)).  Multiplying
// the components 2, 4, 6, ... of every vector by a square root i of -1 maps
// x.y in that metric onto the mostly-minus product of the images
// ((i x^mu)(i y^mu) (-1) = +x^mu y^mu), and the amplitude is built from such
// products alone, so the loaders apply the map and every kernel runs
// unchanged.  Exact in both fields: over C it swaps and negates parts, over
// F_p it is one Montgomery product with i R.
//
// M says where the metric comes from: MetricMM / MetricAlt fix it at compile
// time, MetricRT reads a.metric.  The F_p register kernel branches once, at
// its entry, between a MetricMM and a MetricAlt body: its mostly-minus body
// compiles to faster code that way than a single body with the map chosen at
// run time (0.48 against 0.51 ms per 2^20 points at n = 8, d = 6), although
// the compiler then waits for each load of the alternating body before
// issuing the next, which makes that metric about twice as slow.  The complex
// register kernel and the runtime-n kernels take MetricRT: one body, where
// the map is a select (complex) or, over F_p, one Montgomery product per
// loaded component, with a.ialt for components 2, 4, ... (R in the
// mostly-minus metric) and with R for the others.
enum : int { MetricMM = 0, MetricAlt = 1, MetricRT = 2 };

template <class Fld>
struct Loader;

template <int DL, int L, bool SC>
struct Loader<FpField<DL, L, SC>> {
  template <int M>
  __device__ static int32_t get(const LaunchArgs& a, const void* base, int l, int mu, int64_t q,
                                uint32_t& maxraw) {
    const bool in = mu < a.d;
    const uint32_t x =
        static_cast<const uint32_t*>(base)[((int64_t)l * a.d + (in ? mu : 0)) * a.ld + q];
    const uint32_t xi = in ? x : 0u;
    maxraw = maxraw > xi ? maxraw : xi;
    const uint32_t xc = xi < (uint32_t)a.fp.p ? xi : 0u;
    const bool rot = mu >= 2 && (mu & 1) == 0;
    if constexpr (M == MetricRT) {
      // one product for every component, with R (the conversion, bit for bit:
      // both results are balanced) or with a.ialt: a select between a product
      // and the conversion became a branch around each load, which then
      // waited for every load before issuing the next
      return fp_mul((int32_t)xc, rot ? a.ialt : a.fp.one, a.fp);
    } else {
      int32_t v = fp_from_canonical(xc, a.fp);
      if constexpr (M == MetricAlt) {  // a select, so that the loads stay in one block
        const int32_t w = fp_mul(v, a.ialt, a.fp);
        v = rot ? w : v;
      }
      return v;
    }
  }
};

template <int DL, int L>
struct Loader<C128Field<DL, L>> {
  template <int M>
  __device__ static cplx get(const LaunchArgs& a, const void* base, int l, int mu, int64_t q,
                             uint32_t&) {
    const bool in = mu < a.d;
    const double2 v =
        static_cast<const double2*>(base)[((int64_t)l * a.d + (in ? mu : 0)) * a.ld + q];
    // selects, not branches: an early return here lets the compiler sink each
    // load into a block of its own, which serialises the point's loads.
    // Component 0 is multiplied by i (C128Field holds time components that
    // way), and in the alternating metric so are components 2, 4, 6, ...
    const bool alt = M == MetricAlt || (M == MetricRT && a.metric != 0);
    double re = in ? v.x : 0.0, im = in ? v.y : 0.0;
    const bool rot = mu == 0 || (alt && mu >= 2 && (mu & 1) == 0);  // times i, exactly
    const double r2 = rot ? -im : re, i2 = rot ? re : im;
    return cplx{r2, i2};
  }
};

// ---------------------------------------------------------------------------
// propagator inverses: inv'(S) = 2 / P_S^2, given y(S) = -P_S^2
// ---------------------------------------------------------------------------
template <class Fld, int NP>
struct Inverses {};

template <int DL, int L, bool SC, int NP>
struct Inverses<FpField<DL, L, SC>, NP> {
  // Montgomery batch inversion (Montgomery 1987): one Fermat power for all NP
  // values; a zero anywhere makes the point singular.  inv(s) receives
  // 2/P_S^2 for y(s) = -P_S^2, as the finish of each current expects it.
  //
  // General schedule: products are Montgomery products with R = 2^64 (fp_mul).
  // Small fold constant: products are taken in the Montgomery domain of 2^32
  // (mulp: a b 2^-32, one fold and one 32-bit REDC step), with 1 = 2^32 mod
  // p.  There y(s) = -P^2 R stands for -P^2 2^32, so its inverse comes out as
  // the plain residue -1/P^2, and the final product with the plain residue -2
  // gives 2/P^2 2^-32, the extra 2^-32 that the small-fold finish needs.
  template <class Tab>
  __device__ static bool compute(const FpField<DL, L, SC>& F, int32_t (&y)[NP > 0 ? NP : 1], Tab& inv) {
    if constexpr (NP == 0) {
      return false;
    } else {
      auto mul = [&](int32_t a, int32_t b) {
        if constexpr (SC) return F.mulp(a, b);
        else return fp_mul(a, b, F.k);
      };
      bool zero = false;
      int32_t pre[NP];
#pragma unroll
      for (int s = 0; s < NP; ++s) {
        if (y[s] == 0) { zero = true; y[s] = F.k.one; }
        pre[s] = s == 0 ? y[0] : mul(pre[s - 1], y[s]);
      }
      // a^(p-2) as straight-line code: 31 square-and-select steps, both
      // products formed every step.  A few more products than a loop over the
      // set bits, but the kernel stays one basic block, so the compiler keeps
      // seeing its int32 values as sign-extended 32-bit operands (values
      // carried across a loop were multiplied with the generic 64-bit sequence
      // instead of one v_mad_i64_i32).
      const uint32_t e = (uint32_t)(F.k.p - 2);
      int32_t t = SC ? F.k.c32 : F.k.one;
#pragma unroll
      for (int b = 30; b >= 0; --b) {
        t = mul(t, t);
        const int32_t m = mul(t, pre[NP - 1]);
        t = ((e >> b) & 1u) ? m : t;
      }
      // the factor -2 turns 1/y = -1/P^2 into 2/P^2 for every element.  It
      // is applied as the plain residue 2 (the constant 2 times R^-1), which
      // removes both the 2^32 that lazily reduced scalars leave in the current
      // accumulators and the 2^-32 of the single 32-bit REDC step that
      // finishes each current (FpField::finish_mul32)
      t = mul(t, -2);
#pragma unroll
      for (int s = NP - 1; s >= 0; --s) {
        inv.set(s, s == 0 ? t : mul(t, pre[s - 1]));
        if (s > 0) t = mul(t, y[s]);
      }
      return zero;
    }
  }
};

// ---------------------------------------------------------------------------
// per-point tables that may live in registers or in LDS
// ---------------------------------------------------------------------------
// Store<T, SLOTS, LDS>: SLOTS values of T for this lane (or this point).  In
// register mode a plain array (indexed with compile-time slots after
// unrolling); in LDS mode a [slot][column] array in shared memory, with one
// column per lane (vectors) or per point (scalars shared by the L lanes of a
// point: every lane of the group writes the same value, and the group lies in
// one wavefront, so no barrier is needed).
template <class T, int SLOTS, bool LDS>
struct Store {
  T r[SLOTS > 0 ? SLOTS : 1];
  __device__ __forceinline__ T get(int s) const { return r[s]; }
  __device__ __forceinline__ void set(int s, T v) { r[s] = v; }
};

template <class T, int SLOTS>
struct Store<T, SLOTS, true> {
  T* base;
  int stride;
  __device__ __forceinline__ T get(int s) const { return base[s * stride]; }
  __device__ __forceinline__ void set(int s, T v) { base[s * stride] = v; }
};

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <class Fld, int N, int DL, int L, bool LT = false>
struct Recursion {
  using E = typename Fld::E;
  using S = typename Fld::S;
  using A = typename Fld::A;
  using R = Ranges<N>;
  static constexpr int NCUR = R::ncur;   // non-root currents
  static constexpr int NP = R::nprop;    // propagators

  // LDS footprint of the tables when LT: scalars per point, vector slots per lane
  static constexpr int kScalars = Fld::exact ? 2 * NP + NCUR : NP;
  static constexpr int kVecSlots = (Fld::exact ? N + 1 : N) * DL;

  template <int BLOCK>
  struct Lds {
    S scal[LT ? kScalars : 1][BLOCK / L];
    E vec[LT ? kVecSlots : 1][BLOCK];
  };

  template <class Tab>
  __device__ static void bind(Tab& t, void* base, int stride) {
    if constexpr (LT) {
      t.base = static_cast<decltype(t.base)>(base);
      t.stride = stride;
    }
  }

  template <int BLOCK, int M>
  __device__ static void run(const Fld& F, const LaunchArgs& a, int64_t q, int s, uint32_t& bad,
                             bool& singular, S& result, E (&kroot)[DL], Lds<BLOCK>* lds) {
    constexpr bool kFp = Fld::exact;
    E J[NCUR][DL];
    E epsn[DL];
    // per-point scalars: -Dh(X) for |X| >= 2 (by propagator index; complex:
    // -Dh(X) / L), and on F_p nc(X) = -(P_X . J_X) (by range index) and the
    // propagator inverses
    Store<S, NP, LT> nDh;
    Store<S, kFp ? NCUR : 0, LT> nc;
    Store<S, kFp ? NP : 0, LT> inv;
    // F_p: prefix sums Q_l (exact, so P_S = Q_{j+1} - Q_i); complex: primed
    // momenta k'_l.  Slot l * DL + c.
    Store<E, kVecSlots, LT> mom;
    // complex: primed column P'_{i..j} for the current right end j, built by
    // left-to-right sums exactly as the definition of P_{i,j} reads (no
    // differences of large partial sums)
    E col[kFp ? 1 : N][DL];
    const int mu0 = s * DL;
    if constexpr (LT) {
      const int pcol = (int)(threadIdx.x / L), lcol = (int)threadIdx.x;
      bind(nDh, &lds->scal[0][pcol], BLOCK / L);
      bind(nc, &lds->scal[NP][pcol], BLOCK / L);
      bind(inv, &lds->scal[NP + (kFp ? NCUR : 0)][pcol], BLOCK / L);
      bind(mom, &lds->vec[0][lcol], BLOCK);
    }
    auto Qg = [&](int l, int c) { return mom.get(l * DL + c); };

    // ---- a1: loads; a2: sub-range momenta ----------------------------------
    if constexpr (kFp) {
#pragma unroll
      for (int c = 0; c < DL; ++c) mom.set(c, E{});
    }
    static_for<0, N>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      E k[DL];
#pragma unroll
      for (int c = 0; c < DL; ++c) {
        k[c] = Loader<Fld>::template get<M>(a, a.momenta, l, mu0 + c, q, bad);
        J[R::idx(l, l)][c] = Loader<Fld>::template get<M>(a, a.pols, l, mu0 + c, q, bad);
      }
      k[0] = F.prime0(k[0]);
      if constexpr (kFp) {
        nc.set(R::idx(l, l), F.template ndot<2, true>(k, J[R::idx(l, l)]));  // lazily reduced
        k[0] = F.prime0(k[0]);
#pragma unroll
        for (int c = 0; c < DL; ++c) mom.set((l + 1) * DL + c, F.eadd(Qg(l, c), k[c]));
      } else {
#pragma unroll
        for (int c = 0; c < DL; ++c) mom.set(l * DL + c, k[c]);
      }
    });
#pragma unroll
    for (int c = 0; c < DL; ++c) epsn[c] = Loader<Fld>::template get<M>(a, a.pols, N, mu0 + c, q, bad);

    // ---- a3/a4 (F_p): all propagator denominators, one batched inversion -----
    if constexpr (kFp) {
      int32_t y[NP > 0 ? NP : 1];  // y(S) = -P_S^2
      static_for<2, N>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        static_for<0, N - m + 1>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          constexpr int j = i + m - 1;
          E Pp[DL], P[DL];
          if constexpr (Fld::kSC) {
            // P_S lazily normalised (|slot| <= h + 2^23): 66 units a product
#pragma unroll
            for (int c = 0; c < DL; ++c) P[c] = F.lazy_norm(Qg(j + 1, c) - Qg(i, c));
            unprime(F, P, Pp);
            y[R::pidx(i, j)] = F.template ndot<5>(Pp, P);
          } else {
            primedP<i, j>(F, mom, Pp);
            unprime(F, Pp, P);
            y[R::pidx(i, j)] = F.ndot(Pp, P);
          }
        });
      });
      singular = Inverses<Fld, NP>::compute(F, y, inv);
    } else {
#pragma unroll
      for (int c = 0; c < DL; ++c) col[0][c] = Qg(0, c);
    }

    // ---- a5: the recursion, column by column (right end j), each column from
    // the shortest range up; every range it reads is already final.
    static_for<1, N>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      if constexpr (!kFp) {
        // column j: P'_{i..j} = P'_{i..j-1} + k'_j
        static_for<0, j>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          E kj[DL];
#pragma unroll
          for (int c = 0; c < DL; ++c) kj[c] = Qg(j, c);
#pragma unroll
          for (int c = 0; c < DL; ++c) col[i][c] = F.eadd(col[i][c], kj[c]);
        });
#pragma unroll
        for (int c = 0; c < DL; ++c) col[j][c] = Qg(j, c);
      }
      static_for<0, j>([&](auto ic) {
        constexpr int i = j - 1 - decltype(ic)::value;
        constexpr bool root = (i == 0 && j == N - 1);
        E Pp[DL];
        if constexpr (kFp) {
          lazyP<i, j>(F, mom, Pp);  // unreduced: |slot| <= 2h
        } else {
#pragma unroll
          for (int c = 0; c < DL; ++c) Pp[c] = col[i][c];
        }
        A K[DL];
#pragma unroll
        for (int c = 0; c < DL; ++c) K[c] = F.azero();
        // F_p, small fold constant: bound of K (and of nDacc) in units of
        // 2^54; every loop here is unrolled, so these are compile-time
        // constants and every fold decision is resolved at compile time
        [[maybe_unused]] int uK = 0, uD = 0;

        // three-gluon vertex, A = [i..t], B = [t+1..j]
        S nDsum = F.szero();
        [[maybe_unused]] int64_t nDacc = 0;  // F_p: sum of -(J_A.J_B) * (1/2), unreduced
        [[maybe_unused]] E PA[DL];
        // The LDS operands of a split (complex: k'_t; F_p: Q_{t+1}, c(A),
        // c(B)) are read one split ahead, inside the previous split's
        // scheduling region: with one wave per SIMD the read latency is
        // otherwise exposed at the start of every split.
        // The adjacent-pair terms -Dh(A) J_B and -Dh(B) J_A of the four-gluon
        // vertex share the three-gluon axpys of J_B and J_A (complex, and the
        // small-fold-constant F_p schedule, where the two extra products fit
        // the scalars' budget)
        constexpr bool kMergeDh = !kFp || Fld::kSC;
        struct SplitLds {
          E v[DL];
          S ca, cb;  // F_p: c(A), c(B)
          // merged schedule: -Dh(A), -Dh(B) where that part has two legs or
          // more (complex: their L-th parts, see ndot_from)
          S da, db;
        };
        auto lds_of = [&](auto tc) {
          constexpr int t = decltype(tc)::value;
          SplitLds o;
#pragma unroll
          for (int c = 0; c < DL; ++c) o.v[c] = kFp ? Qg(t + 1, c) : Qg(t, c);
          if constexpr (kFp) {
            o.ca = nc.get(R::idx(i, t));
            o.cb = nc.get(R::idx(t + 1, j));
          }
          if constexpr (kMergeDh && t > i) o.da = nDh.get(R::pidx(i, t));
          if constexpr (kMergeDh && t + 1 < j) o.db = nDh.get(R::pidx(t + 1, j));
          return o;
        };
        SplitLds next = lds_of(std::integral_constant<int, i>{});
        static_for<i, j>([&](auto tc) {
          constexpr int t = decltype(tc)::value;
          constexpr int ia = R::idx(i, t), ib = R::idx(t + 1, j);
          const SplitLds cur = next;
          if constexpr (t + 1 < j) next = lds_of(std::integral_constant<int, t + 1>{});
          // -(J_A.J_B); F_p: lazily reduced (it only multiplies balanced values)
          const S nDm = F.template ndot_u<kFp>(J[ia], J[ib]);
          if constexpr (kFp) {
            // P_B.J_A = P_S.J_A - c(A),  P_A.J_B = P_S.J_B - c(B),
            // P_A - P_B = 2 Q_{t+1} - Q_i - Q_{j+1}
            // lazy P_S slots, lazy stored P_X.J_X, lazily reduced results
            // -(P_B.J_A), merged: -(P_B.J_A) + Dh(A)
            S nc2, nc3;
            if constexpr (kMergeDh && t > i) nc2 = F.template ndot_sub2<4, 3, true>(Pp, J[ia], cur.ca, cur.da);
            else nc2 = F.template ndot_sub<4, 3, true>(Pp, J[ia], cur.ca);
            // -(P_A.J_B), merged: -(P_A.J_B) - Dh(B)
            if constexpr (kMergeDh && t + 1 < j)
              nc3 = F.template ndot_sub2<4, 3, true>(Pp, J[ib], cur.cb, F.sneg(cur.db));
            else nc3 = F.template ndot_sub<4, 3, true>(Pp, J[ib], cur.cb);
            F.template kaxpy<Fld::kPLazy>(K, uK, F.sneg(nDm), cur.v);          // times Q_{t+1}
            F.template kaxpy<Fld::kPLazy>(K, uK, F.sneg(nc2), J[ib]);
            F.template kaxpy<Fld::kPLazy>(K, uK, nc3, J[ia]);
            F.fixed_fold(K);
          } else {
#pragma unroll
            for (int c = 0; c < DL; ++c) PA[c] = (t == i) ? cur.v[c] : F.eadd(PA[c], cur.v[c]);
            // -(P_B.J_A) + Dh(A) (negated below) and -(P_A.J_B) - Dh(B)
            S n2, n3;
            if constexpr (t > i) n2 = F.ndot_from(col[t + 1], J[ia], cneg(cur.da));
            else n2 = F.ndot(col[t + 1], J[ia]);
            if constexpr (t + 1 < j) n3 = F.ndot_from(PA, J[ib], cur.db);
            else n3 = F.ndot(PA, J[ib]);
            // (1/2)(J_A.J_B)(P_A - P_B) = (J_A.J_B) P_A - (1/2)(J_A.J_B) P_S:
            // the P_S part is summed over the splits and added once
            F.axpy(K, F.sneg(nDm), PA);
            F.axpy(K, F.sneg(n2), J[ib]);
            F.axpy(K, n3, J[ia]);
          }
          if constexpr (kFp) {
            if constexpr (Fld::kSC) {
              F.template kmad<Fld::kPLazy>(nDacc, uD, nDm, F.k.inv2);
            } else {
              // products below 3 half-units (lazy nDm times balanced 1/2): fold
              // before every third one after the first three
              if constexpr (t > i && (t - i) % 3 == 0) nDacc = fp_fold(nDacc, F.k);
              nDacc = mad64(nDm, F.k.inv2, nDacc);
            }
          } else {
            nDsum = accumulate_scalar(F, nDsum, nDm);
          }
          split_barrier();
        });
        S nDhS;
        if constexpr (kFp) {
          nDhS = fp_redc2(fp_fold(nDacc, F.k), F.k);
          // -Dh(S) (Q_i + Q_{j+1}), the two prefix sums added unreduced (|.| <= 2h)
          E QQ[DL];
#pragma unroll
          for (int c = 0; c < DL; ++c) QQ[c] = Qg(i, c) + Qg(j + 1, c);
          F.template kaxpy<Fld::kPBalDiff>(K, uK, nDhS, QQ);
          F.fixed_fold(K);
        } else {
          // stored as its L-th part (the splits that read it start their
          // lanes' partial dot products from it)
          nDhS = {(0.5 / L) * nDsum.re, (0.5 / L) * nDsum.im};
          F.axpy(K, cplx{0.5 * nDsum.re, 0.5 * nDsum.im}, Pp);
        }
        if constexpr (!root) nDh.set(R::pidx(i, j), nDhS);

        // four-gluon vertex: sum (J_A.J_C) J_B, then the Dh terms
        static_for<i, j - 1>([&](auto sc) {
          constexpr int s1 = decltype(sc)::value;
          static_for<s1 + 1, j>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            const S ne = F.template ndot_u<kFp>(J[R::idx(i, s1)], J[R::idx(t + 1, j)]);  // F_p: lazy
            F.template kaxpy<Fld::kPLazy>(K, uK, F.sneg(ne), J[R::idx(s1 + 1, t)]);
            constexpr int qn = v4_index<i, j>(s1, t);
            // F_p, general schedule: lazy scalars give products below 3
            // half-units: fold every third
            if constexpr (qn % 3 == 2) F.fixed_fold(K);
            split_barrier();
          });
        });
        F.fixed_fold(K);
        if constexpr (!kMergeDh) {
          static_for<i + 1, j>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            F.template kaxpy<Fld::kPBal>(K, uK, nDh.get(R::pidx(i, t)), J[R::idx(t + 1, j)]);
            if constexpr ((t - i) % 5 == 4) F.fixed_fold(K);
          });
          F.fixed_fold(K);
          static_for<i, j - 1>([&](auto sc) {
            constexpr int s1 = decltype(sc)::value;
            F.template kaxpy<Fld::kPBal>(K, uK, nDh.get(R::pidx(s1 + 1, j)), J[R::idx(i, s1)]);
            if constexpr ((s1 - i) % 5 == 4) F.fixed_fold(K);
          });
        }

        if constexpr (!root) {
          // J(S) = K' * 2/P_S^2
          S inv2;
          if constexpr (kFp) {
            inv2 = inv.get(R::pidx(i, j));
          } else {
            E P[DL];
            unprime(F, Pp, P);
            const S y = F.ndot(Pp, P);  // -P^2
            inv2 = c_inverse_times(y, -2.0, singular);
          }
          constexpr int id = R::idx(i, j);
          if constexpr (kFp) {
#pragma unroll
            for (int c = 0; c < DL; ++c) J[id][c] = F.finish_mul32(K[c], inv2);
            nc.set(id, F.template ndot<4, true>(Pp, J[id]));  // lazily reduced
          } else {
#pragma unroll
            for (int c = 0; c < DL; ++c) J[id][c] = F.mul(F.finish(K[c]), inv2);
          }
        } else {
          // a6: returns -(eps_n . K'); the amplitude is M = 2 eps_n . K'
          E Kf[DL];
#pragma unroll
          for (int c = 0; c < DL; ++c) Kf[c] = F.finish(K[c]);
          result = F.ndot_u(epsn, Kf);
#pragma unroll
          for (int c = 0; c < DL; ++c) kroot[c] = Kf[c];
        }
      });
    });
  }

  __device__ static __forceinline__ void unprime(const Fld& F, const E (&Pp)[DL], E (&P)[DL]) {
#pragma unroll
    for (int c = 0; c < DL; ++c) P[c] = Pp[c];
    P[0] = F.prime0(Pp[0]);
  }

  // Keeps the scheduler from interleaving many splits at once: the current
  // table is already most of the register file, so unbounded interleaving
  // turns into spills.
  __device__ static __forceinline__ void split_barrier() {
#if BG_SPLIT_BARRIER
    __builtin_amdgcn_sched_barrier(BG_SPLIT_BARRIER_MASK);
#endif
  }

  // primed P_S = Q_{j+1} - Q_i as plain int32 differences of balanced values
  // (|slot| <= 2h < 2^31; a product with a balanced value is below 2^61), with
  // the time slot negated (F_p)
  template <int i, int j, class Tab>
  __device__ static __forceinline__ void lazyP(const Fld& F, const Tab& Q, E (&P)[DL]) {
#pragma unroll
    for (int c = 0; c < DL; ++c) P[c] = Q.get((j + 1) * DL + c) - Q.get(i * DL + c);
    P[0] = F.prime0(P[0]);
  }

  // primed P_S = Q_{j+1} - Q_i with the time slot negated (F_p)
  template <int i, int j, class Tab>
  __device__ static __forceinline__ void primedP(const Fld& F, const Tab& Q, E (&P)[DL]) {
#pragma unroll
    for (int c = 0; c < DL; ++c) P[c] = F.esub(Q.get((j + 1) * DL + c), Q.get(i * DL + c));
    P[0] = F.prime0(P[0]);
  }

  // compile-time position of the V4 split (s, t) of [i..j] in enumeration order
  template <int i, int j>
  static constexpr int v4_index(int s1, int t) {
    int q = 0;
    for (int a = i; a < j - 1; ++a)
      for (int b = a + 1; b < j; ++b) {
        if (a == s1 && b == t) return q;
        ++q;
      }
    return q;
  }

  __device__ static __forceinline__ S accumulate_scalar(const Fld& F, S acc, S x) {
    if constexpr (Fld::exact) return fp_add(acc, x, F.k);
    else return cadd(acc, x);
  }
  __device__ static __forceinline__ S half_scalar(const Fld& F, S x) {
    if constexpr (Fld::exact) return fp_mul(x, F.k.inv2, F.k);
    else return {0.5 * x.re, 0.5 * x.im};
  }
  // f / y for complex y (f real); flags an exact zero
  __device__ static __forceinline__ cplx c_inverse_times(cplx y, double f, bool& singular) {
    const double den = __builtin_fma(y.re, y.re, y.im * y.im);
    singular |= (y.re == 0.0 && y.im == 0.0);
    // 1/den from the hardware reciprocal and two Newton steps (on the
    // residual e = 1 - den r, each step squares the relative error), then
    // times f: six instructions against the eleven of an IEEE division, the
    // same results on 2^17 random points
    double r = __builtin_amdgcn_rcp(den);
    double e = __builtin_fma(-den, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-den, r, 1.0);
    r = __builtin_fma(r, e, r) * f;
    return {y.re * r, -y.im * r};
  }
};

// W = minimum waves per SIMD the register allocation must allow (1: the whole
// register file for one wave; 2: at most 256 registers per lane).
template <class Fld, int N, int DL, int L, int BLOCK, bool LT, int W>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(W)))
void bg_recursion_kernel(LaunchArgs a) {
  using Rec = Recursion<Fld, N, DL, L, LT>;
  __shared__ typename Rec::template Lds<BLOCK> lds;
  const int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int s = (int)(g % L);
  const int64_t q0 = g / L;
  const bool valid = q0 < a.npts;
  const int64_t q = valid ? q0 : a.npts - 1;  // tail groups recompute the last point
  uint32_t bad = 0;
  bool singular = false;
  typename Fld::S res;
  typename Fld::E kroot[DL];
  if constexpr (Fld::exact) {
    Fld F(a.fp, s);
    if (a.metric != 0) Rec::template run<BLOCK, MetricAlt>(F, a, q, s, bad, singular, res, kroot, &lds);
    else Rec::template run<BLOCK, MetricMM>(F, a, q, s, bad, singular, res, kroot, &lds);
    if constexpr (L > 1)
      bad = group_sum<L>(bad, [](uint32_t x, uint32_t y) { return x > y ? x : y; },
                         [](auto ctrl, uint32_t v) { return dpp_u32<decltype(ctrl)::value>(v); });
    bad = bad >= (uint32_t)a.fp.p ? 1u : 0u;
    const uint8_t st = bad ? PT_BADRESIDUE : (singular ? PT_SINGULAR : PT_OK);
    if (a.cur) {
      // root current K = 2 K'; kroot carries R^-3 (degree n - 1 in eps, 4 - n
      // in k) and the accumulator's 2^32: one product with R^3 2^-32 restores it
      if (valid) {
#pragma unroll
        for (int c = 0; c < DL; ++c) {
          const int mu = s * DL + c;
          if (mu < a.d) {
            uint32_t v = 0xFFFFFFFFu;
            if (st == PT_OK) {
              const int32_t m = fp_mul(kroot[c], a.fp.r3s, a.fp);
              v = fp_to_canonical(fp_add(m, m, a.fp), a.fp);
            }
            static_cast<uint32_t*>(a.cur)[(int64_t)mu * a.ld + q] = v;
          }
        }
        if (a.status && s == 0) a.status[q] = st;
      }
    } else if (valid && s == 0) {
      uint32_t outv = 0xFFFFFFFFu;
      if (st == PT_OK) {
        // res = -(eps_n . K') in Montgomery form of a value scaled by R^-4,
        // times the 2^32 that the root accumulator carries; M = 2 eps_n . K'
        // = res * (-2), times R^4 2^-32 to undo both scalings.
        int32_t m = fp_mul(res, a.fp.r4s, a.fp);
        m = fp_sub(0, fp_add(m, m, a.fp), a.fp);     // * (-2)
        outv = fp_to_canonical(m, a.fp);
      }
      static_cast<uint32_t*>(a.out)[q] = outv;
      if (a.status) a.status[q] = st;
    }
  } else {
    Fld F(s);
    Rec::template run<BLOCK, MetricRT>(F, a, q, s, bad, singular, res, kroot, &lds);
    if (a.cur) {
      if (valid) {
#pragma unroll
        for (int c = 0; c < DL; ++c) {
          const int mu = s * DL + c;
          if (mu < a.d) {
            // component 0 back from its factor i: K^0 = -i (i K^0)
            const cplx k = mu == 0 ? cplx{kroot[c].im, -kroot[c].re} : kroot[c];
            double2 o;
            o.x = singular ? __builtin_nan("") : 2.0 * k.re;
            o.y = singular ? __builtin_nan("") : 2.0 * k.im;
            static_cast<double2*>(a.cur)[(int64_t)mu * a.ld + q] = o;
          }
        }
        if (a.status && s == 0) a.status[q] = singular ? PT_SINGULAR : PT_OK;
      }
    } else if (valid && s == 0) {
      double2 o;
      if (singular) {
        o.x = __builtin_nan("");
        o.y = __builtin_nan("");
      } else {
        o.x = -2.0 * res.re;
        o.y = -2.0 * res.im;
      }
      static_cast<double2*>(a.out)[q] = o;
      if (a.status) a.status[q] = singular ? PT_SINGULAR : PT_OK;
    }
  }
}

}  // namespace bg
