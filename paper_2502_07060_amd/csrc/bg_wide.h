// Berends-Giele recursion for large n (paper Sec. 2.2) with a group of G
// lanes per phase-space point and the point's current table shared in LDS.
//
// One lane per point (bg_generic.h) needs the whole table per lane, so only a
// handful of points fit a CU at n >= 9.  Here the G lanes of a group split the
// work of one point instead.  Ranges of one length m depend only on shorter
// ranges, so the recursion advances length by length; within a length, the
// work items are (range S = [i..j], cut c) for i <= c < j:
//
//   the three-gluon split A = [i..c] | B = [c+1..j],
//   every four-gluon split [i..c] | [c+1..t] | [t+1..j] (c < t < j),
//   the two adjacent-pair terms of the four-gluon vertex that pair J_A or
//   J_B with the stored -D/2 of the other part (see bg_kernel.h),
//
// each item summing its contribution to K'(S) over the full d components in
// one lane (no cross-lane dot products).  With G = 16 (and with G = 32 where
// the launch asks for it, at n = 14) the cuts c and i + j - 1 - c form one
// item, which evens out the number of four-gluon splits per item.  Items are dealt to the lanes in rounds of G; after each
// round the lane that owns S (lane i) adds the round's partial sums of S, in
// cut order, to its accumulator, so the result does not depend on timing.
// The owner then finishes S: J(S) = 2 K'(S) / P_S^2 into the LDS table, or
// at the root M = 2 eps_n . K'.
//
// Same identities as the register kernel; the sum over splits is taken in
// item order instead of split order, which changes only the rounding of the
// complex path.  F_p propagator inverses: each lane inverts its share of the
// denominators with one batched inversion and one Fermat power.
//
// Component split (complex).  With Fld = C128Field<DL, LC>, LC > 1, each work
// item belongs to LC adjacent lanes that hold DL = DMAX / LC components each
// and sum dot products over DPP: LC times the lanes per point for the same
// LDS footprint, which is what limits how many points a CU holds at large n.
//
// LDS access.  A lane reads whole table rows, with 16-byte reads (complex
// elements are 16 bytes; F_p rows when they start on 16-byte boundaries).
// The lanes of a wave read rows of unrelated ranges at once, so a row stride
// that is a multiple of 64 bytes (complex d = 4 or 8) sends most of them to
// the same banks; the padded layouts round a row up to an odd number of
// 16-byte units.  Complex sub-range momenta are direct left-to-right sums of
// the legs (no prefix differences); a pair item reads each leg of S once for
// both of its cuts.
#pragma once

#include "bg_generic.h"

namespace bg {

template <class Fld, int DMAX, int G, bool PAD>
struct WideLayout {
  using E = typename Fld::E;
  using S = typename Fld::S;
  using A = typename Fld::A;
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
    unsigned J, mom, epsn, nDh, nc, inv, part, pscal, flags, total;
  };
  __host__ __device__ static int ncur(int N) { return N * (N + 1) / 2 - 1; }
  __host__ __device__ static unsigned up16(size_t x) { return (unsigned)((x + 15) / 16 * 16); }
  // per-point LDS offsets (bytes): current table [range][component], momenta
  // (F_p: prefix sums Q_0..Q_N; complex: primed k'_0..k'_{N-1}) [leg][component],
  // eps_n, scalars by range index, one partial K [lane][component] and one
  // scalar per lane, flags.  A vector is contiguous, so a lane reads it with
  // wide LDS loads.
  __host__ __device__ static Off offsets(int N) {
    Off o{};
    unsigned x = 0;
    o.J = x;      x += up16((size_t)ncur(N) * kS * sizeof(E));
    o.mom = x;    x += up16((size_t)(N + 1) * kS * sizeof(E));
    o.epsn = x;   x += up16((size_t)DMAX * sizeof(E));
    o.nDh = x;    x += up16((size_t)ncur(N) * sizeof(S));
    o.nc = x;     x += kFp ? up16((size_t)ncur(N) * sizeof(S)) : 0u;
    o.inv = x;    x += kFp ? up16((size_t)ncur(N) * sizeof(S)) : 0u;
    o.part = x;   x += up16((size_t)G * kS * sizeof(A));  // one row per item slot
    o.pscal = x;  x += up16((size_t)G * sizeof(S));
    o.flags = x;  x += 16;
    o.total = x;
    return o;
  }
};

// The G lanes of a group lie in one wavefront (G divides 64), so a group needs
// no workgroup barrier: waiting for this wave's LDS operations and keeping
// the compiler from moving LDS accesses across the point is enough.
__device__ __forceinline__ void group_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
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
  // With 16 items per point an item always takes a pair of cuts; with 32 the
  // launch chooses (LaunchArgs::wide_pairs): pairs keep every length of
  // n = 14 within one round of 32 items, single cuts are more items of
  // shorter four-gluon loops; with 64, single cuts
  static constexpr bool kPairsAlways = G < 32;
  static constexpr bool kPairsMaybe = G <= 32;

  E* Jt;
  E* Mt;
  E* En;
  S* nDht;
  S* nct;
  S* invt;
  A* part;
  S* pscal;
  unsigned* flags;
  int N, g, s, ln, co;  // item slot, component part, lane in the point, first component

  __device__ WideRecursion(char* base, int N_, int ln_)
      : N(N_), g(ln_ / LC), s(ln_ % LC), ln(ln_), co((ln_ % LC) * DL) {
    const auto o = Lay::offsets(N);
    Jt = reinterpret_cast<E*>(base + o.J);
    Mt = reinterpret_cast<E*>(base + o.mom);
    En = reinterpret_cast<E*>(base + o.epsn);
    nDht = reinterpret_cast<S*>(base + o.nDh);
    nct = reinterpret_cast<S*>(base + o.nc);
    invt = reinterpret_cast<S*>(base + o.inv);
    part = reinterpret_cast<A*>(base + o.part);
    pscal = reinterpret_cast<S*>(base + o.pscal);
    flags = reinterpret_cast<unsigned*>(base + o.flags);
  }

  __device__ __forceinline__ int rid(int i, int j) const { return range_idx(N, i, j); }
  __device__ __forceinline__ E& Jat(int r, int c) const { return Jt[r * kS + c]; }
  __device__ __forceinline__ E& Mat(int l, int c) const { return Mt[l * kS + c]; }
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
  // primed P_S (F_p: reduced, from prefix sums; complex: left-to-right sum of k')
  __device__ __forceinline__ void primedP(const Fld& F, int i, int j, E (&P)[DL]) const {
    if constexpr (kFp) {
      E a[DL], b[DL];
      loadM(j + 1, a);
      loadM(i, b);
#pragma unroll
      for (int c = 0; c < DL; ++c) P[c] = F.esub(a[c], b[c]);
      P[0] = F.prime0(P[0]);
    } else {
      loadM(i, P);
      for (int l = i + 1; l <= j; ++l) {
        E t[DL];
        loadM(l, t);
#pragma unroll
        for (int c = 0; c < DL; ++c) P[c] = F.eadd(P[c], t[c]);
      }
    }
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
  // complex: the primed momenta of both cuts c1 <= c2 of S = [i..j] in one
  // pass over the legs, each leg read once and added to the sums it belongs
  // to, every sum still taken left to right:
  //   legs i..c1 -> A1 (and A2, which starts as A1);  c1+1..c2 -> B1, A2;
  //   c2+1..j -> B1, B2
  __device__ __forceinline__ void pair_momenta(int i, int j, int c1, int c2, E (&A1)[DL], E (&B1)[DL],
                                               E (&A2)[DL], E (&B2)[DL]) const {
#pragma unroll
    for (int c = 0; c < DL; ++c) A1[c] = B1[c] = B2[c] = cplx{0.0, 0.0};
    int l = i;
    for (; l <= c1; ++l) {
      E t[DL];
      loadM(l, t);
#pragma unroll
      for (int c = 0; c < DL; ++c) A1[c] = cadd(A1[c], t[c]);
    }
#pragma unroll
    for (int c = 0; c < DL; ++c) A2[c] = A1[c];
    for (; l <= c2; ++l) {
      E t[DL];
      loadM(l, t);
#pragma unroll
      for (int c = 0; c < DL; ++c) {
        B1[c] = cadd(B1[c], t[c]);
        A2[c] = cadd(A2[c], t[c]);
      }
    }
    for (; l <= j; ++l) {
      E t[DL];
      loadM(l, t);
#pragma unroll
      for (int c = 0; c < DL; ++c) {
        B1[c] = cadd(B1[c], t[c]);
        B2[c] = cadd(B2[c], t[c]);
      }
    }
  }

  // ---- loads: eps into the table, momenta, eps_n; F_p prefix sums --------
  __device__ void load(const Fld& F, const LaunchArgs& a, int64_t q, uint32_t& bad) {
    const int rows = (2 * N + 1) * DMAX;  // eps_0..eps_N, k_0..k_{N-1}
    for (int r = ln; r < rows; r += G * LC) {
      const int which = r / DMAX, c = r % DMAX;
      if (which <= N) {
        const E e = Loader<Fld>::template get<MetricRT>(a, a.pols, which, c, q, bad);
        if (which < N) Jat(rid(which, which), c) = e;
        else En[c] = e;
      } else {
        const int l = which - N - 1;
        E k = Loader<Fld>::template get<MetricRT>(a, a.momenta, l, c, q, bad);
        if constexpr (kFp) {
          Mat(l + 1, c) = k;  // raw k_l, summed below
        } else {
          if (c == 0) k = F.prime0(k);
          Mat(l, c) = k;
        }
      }
    }
    if (ln == 0) *flags = 0u;
    group_sync();
    if constexpr (kFp) {
      if (g < DMAX) {  // prefix sums, one component per lane
        E acc{};
        Mat(0, g) = acc;
        for (int l = 0; l < N; ++l) {
          acc = F.eadd(acc, Mat(l + 1, g));
          Mat(l + 1, g) = acc;
        }
      }
      group_sync();
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

  // ---- one work item: contributions of cut c to K'(S), S = [i..j] ---------
  // cut3: the three-gluon split [i..c] | [c+1..j] and the adjacent-pair terms
  // of the four-gluon vertex that involve this cut; cut4 below adds the
  // four-gluon splits of one or two cuts.
  // F_p: Pp holds P_S as unreduced differences, nDs accumulates -(J_A.J_B) / 2
  // as an int64 sum of products; complex: PA, PB are the primed P_A, P_B
  // (Pp unused), nDs sums -(J_A.J_B).
  template <class NDS>
  __device__ void cut3(const Fld& F, int i, int j, int c, const E (&Pp)[DL], const E (&PA)[DL],
                      const E (&PB)[DL], A (&K)[DL], NDS& nDs) const {
    E JA[DL], JB[DL];
    const int ra = rid(i, c), rb = rid(c + 1, j);
    loadJ(ra, JA);
    loadJ(rb, JB);
    const S nDm = F.ndot_u(JA, JB);  // -(J_A . J_B)
    if constexpr (kFp) {
      E Qt[DL];
      loadM(c + 1, Qt);
      const S nc2 = F.template ndot_sub<4>(Pp, JA, nct[ra]);   // -(P_B . J_A)
      const S nc3 = F.template ndot_sub<4>(Pp, JB, nct[rb]);   // -(P_A . J_B)
      F.axpy(K, F.sneg(nDm), Qt);
      F.axpy(K, F.sneg(nc2), JB);
      F.axpy(K, nc3, JA);
      F.fold(K);
      nDs = mad64(nDm, F.k.inv2, nDs);  // at most two terms per item
    } else {
      E v[DL];
      const S n2 = F.ndot(PB, JA);
      const S n3 = F.ndot(PA, JB);
#pragma unroll
      for (int x = 0; x < DL; ++x) v[x] = F.esub(PA[x], PB[x]);
      v[0] = F.prime0(v[0]);  // P_A - P_B
      F.axpy(K, cplx{-0.5 * nDm.re, -0.5 * nDm.im}, v);
      F.axpy(K, F.sneg(n2), JB);
      F.axpy(K, n3, JA);
      nDs = cadd(nDs, nDm);
    }
    // adjacent-pair terms of the four-gluon vertex that involve this cut
    if (c >= i + 1) F.axpy(K, nDht[ra], JB);
    if (c <= j - 2) F.axpy(K, nDht[rb], JA);
    F.fold(K);
  }

  // four-gluon splits [i..c] | [c+1..t] | [t+1..j] of cut c1 (j - c1 - 1 of
  // them), then of cut c2 (j - c2 - 1; none when c2 == c1), in one loop: the
  // two cuts of a pair item have m - 2 splits together, so every lane of a
  // round runs the same number of iterations (two loops back to back would
  // run m - 2 + m/2 - 1, with lanes masked off).  Range indices advance
  // incrementally: with e = (right end - left end) of a range, extending
  // [c+1..t] to [c+1..t+1] adds N - e, and shrinking [t+1..j] to [t+2..j]
  // adds e - N (from the index formula of range_idx).
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

  __device__ void run(const Fld& F, const LaunchArgs& a, int64_t q, S& result, E (&kroot)[DL]) {
    uint32_t bad = 0;
    bool singular = false;
    load(F, a, q, bad);
    inverses(F, singular);
    group_sync();
    // complex: lane g owns [g..g+m-1] at every length m while g < N - m + 1,
    // so it keeps that range's primed momentum as a running left-to-right sum
    // (the same additions in the same order as summing the legs afresh)
    [[maybe_unused]] E Pown[DL];
    if constexpr (!kFp) {
      if (g < N) loadM(g, Pown);
    }

    const bool pairs = kPairsAlways || (kPairsMaybe && a.wide_pairs != 0);
    for (int m = 2; m <= N; ++m) {
      const int nr = N - m + 1;                 // ranges of length m: i = 0 .. nr-1
      const int per = pairs ? m / 2 : m - 1;    // items per range
      const int items = nr * per;
      const bool own = g < nr;
      const int oi = g, oj = g + m - 1;         // the range this lane owns
      A K[DL];
#pragma unroll
      for (int c = 0; c < DL; ++c) K[c] = F.azero();
      S nDsum = F.szero();
      for (int k0 = 0; k0 < items; k0 += G) {
        const int k = k0 + g;
        if (k < items) {
          const int i = k / per, u = k % per, j = i + m - 1;
          E Pp[DL];
          if constexpr (kFp) lazyP(F, i, j, Pp);
          A Kp[DL];
#pragma unroll
          for (int c = 0; c < DL; ++c) Kp[c] = F.azero();
          const int c1 = i + u, c2 = pairs ? j - 1 - u : c1;
          if constexpr (kFp) {
            int64_t nDs = 0;
            cut3(F, i, j, c1, Pp, Pp, Pp, Kp, nDs);
            if (pairs && c2 != c1) cut3(F, i, j, c2, Pp, Pp, Pp, Kp, nDs);
            cut4(F, i, j, c1, c2, Kp);
            pscal[g] = fp_redc2(fp_fold(nDs, F.k), F.k);  // -(sum of J_A.J_B) / 2
          } else {
            S nDs = F.szero();
            if (pairs) {
              E PA1[DL], PB1[DL], PA2[DL], PB2[DL];
              pair_momenta(i, j, c1, c2, PA1, PB1, PA2, PB2);
              cut3(F, i, j, c1, Pp, PA1, PB1, Kp, nDs);
              if (c2 != c1) cut3(F, i, j, c2, Pp, PA2, PB2, Kp, nDs);
            } else {
              E PA[DL], PB[DL];
              primedP(F, i, c1, PA);
              primedP(F, c1 + 1, j, PB);
              cut3(F, i, j, c1, Pp, PA, PB, Kp, nDs);
            }
            cut4(F, i, j, c1, c2, Kp);
            if (s == 0) pscal[g] = nDs;
          }
#pragma unroll
          for (int c = 0; c < DL; ++c) part[g * kS + co + c] = Kp[c];
        }
        group_sync();
        if (own) {
          // this round's items of the owned range, in item (= cut) order
          const int lo = max(k0, oi * per), hi = min(k0 + G, (oi + 1) * per);
          for (int kk = lo; kk < hi; ++kk) {
            const int slot = kk - k0;
#pragma unroll
            for (int c = 0; c < DL; ++c) K[c] = add_acc(F, K[c], part[slot * kS + co + c]);
            nDsum = Rec::accumulate_scalar(F, nDsum, pscal[slot]);
          }
        }
        group_sync();
      }
      if (own) {
        const bool root = (m == N);
        S nDhS;
        E Pp[DL];
        if constexpr (kFp) {
          nDhS = nDsum;  // the items' sums already carry the factor 1/2
          lazyP(F, oi, oj, Pp);
          // -Dh(S) (Q_i + Q_{j+1}), the prefix sums added unreduced (|.| <= 2h)
          E QQ[DL];
#pragma unroll
          for (int c = 0; c < DL; ++c) QQ[c] = Mat(oi, co + c) + Mat(oj + 1, co + c);  // once per range
          F.axpy(K, nDhS, QQ);
          F.fold(K);
        } else {
          nDhS = Rec::half_scalar(F, nDsum);
          E t[DL];
          loadM(oj, t);
#pragma unroll
          for (int c = 0; c < DL; ++c) {
            Pown[c] = F.eadd(Pown[c], t[c]);
            Pp[c] = Pown[c];
          }
        }
        if (!root) {
          const int id = rid(oi, oj);
          nDht[id] = nDhS;
          E Jn[DL];
          if constexpr (kFp) {
            const S inv2 = invt[id];
#pragma unroll
            for (int c = 0; c < DL; ++c) {
              Jn[c] = F.finish_mul32(K[c], inv2);
              Jat(id, co + c) = Jn[c];
            }
            nct[id] = F.template ndot<4>(Pp, Jn);
          } else {
            E Pu[DL];
#pragma unroll
            for (int c = 0; c < DL; ++c) Pu[c] = Pp[c];
            Pu[0] = F.prime0(Pp[0]);
            const S y = F.ndot(Pp, Pu);
            const S inv2 = Rec::c_inverse_times(y, -2.0, singular);
#pragma unroll
            for (int c = 0; c < DL; ++c) {
              Jn[c] = F.mul(F.finish(K[c]), inv2);
              Jat(id, co + c) = Jn[c];
            }
          }
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
      group_sync();
    }
    // per-point flags: bit 0 bad residue (F_p), bit 1 singular
    unsigned fl = singular ? 2u : 0u;
    if constexpr (kFp) fl |= bad >= (uint32_t)F.k.p ? 1u : 0u;
    if (fl) atomicOr(flags, fl);
    group_sync();
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
