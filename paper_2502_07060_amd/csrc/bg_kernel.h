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
// small sub-range momenta independent of the size of the partial sums.
#pragma once

#include "bg_common.h"
#include "bg_fields.h"

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
};

// ---------------------------------------------------------------------------
// loads
// ---------------------------------------------------------------------------
template <class Fld>
struct Loader;

template <int DL, int L>
struct Loader<FpField<DL, L>> {
  __device__ static int32_t get(const LaunchArgs& a, const void* base, int l, int mu, int64_t q,
                                uint32_t& bad) {
    if (mu >= a.d) return 0;
    uint32_t x = static_cast<const uint32_t*>(base)[((int64_t)l * a.d + mu) * a.ld + q];
    bad |= (x >= (uint32_t)a.fp.p) ? 1u : 0u;
    return fp_from_canonical(x < (uint32_t)a.fp.p ? x : 0u, a.fp);
  }
};

template <int DL, int L>
struct Loader<C128Field<DL, L>> {
  __device__ static cplx get(const LaunchArgs& a, const void* base, int l, int mu, int64_t q,
                             uint32_t&) {
    if (mu >= a.d) return {0.0, 0.0};
    const double2 v = static_cast<const double2*>(base)[((int64_t)l * a.d + mu) * a.ld + q];
    return {v.x, v.y};
  }
};

// ---------------------------------------------------------------------------
// propagator inverses: inv'(S) = 2 / P_S^2, given y(S) = -P_S^2
// ---------------------------------------------------------------------------
template <class Fld, int NP>
struct Inverses {};

template <int DL, int L, int NP>
struct Inverses<FpField<DL, L>, NP> {
  int32_t inv[NP > 0 ? NP : 1];
  // Montgomery batch inversion (Montgomery 1987): one Fermat power for all NP
  // values; a zero anywhere makes the point singular.
  __device__ bool compute(const FpField<DL, L>& F, int32_t (&y)[NP > 0 ? NP : 1]) {
    if constexpr (NP == 0) {
      return false;
    } else {
      bool zero = false;
      int32_t pre[NP];
#pragma unroll
      for (int s = 0; s < NP; ++s) {
        if (y[s] == 0) { zero = true; y[s] = F.k.one; }
        pre[s] = s == 0 ? y[0] : fp_mul(pre[s - 1], y[s], F.k);
      }
      // the factor -2 turns 1/y = -1/P^2 into 2/P^2 for every element
      int32_t t = fp_pow(pre[NP - 1], (uint32_t)(F.k.p - 2), F.k);
      t = fp_mul(t, -F.k.two, F.k);
#pragma unroll
      for (int s = NP - 1; s >= 0; --s) {
        inv[s] = s == 0 ? t : fp_mul(t, pre[s - 1], F.k);
        if (s > 0) t = fp_mul(t, y[s], F.k);
      }
      return zero;
    }
  }
  __device__ __forceinline__ int32_t get(int s) const { return inv[s]; }
};

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <class Fld, int N, int DL, int L>
struct Recursion {
  using E = typename Fld::E;
  using S = typename Fld::S;
  using A = typename Fld::A;
  using R = Ranges<N>;
  static constexpr int NCUR = R::ncur;   // non-root currents
  static constexpr int NP = R::nprop;    // propagators

  __device__ static void run(const Fld& F, const LaunchArgs& a, int64_t q, int s, uint32_t& bad,
                             bool& singular, S& result) {
    constexpr bool kFp = Fld::exact;
    E J[NCUR][DL];
    S nDh[NCUR];                 // -Dh(X) for |X| >= 2 (indexed by range index)
    E epsn[DL];
    // F_p: prefix sums Q_l and nc(X) = -(P_X . J_X); exact, so P_S = Q_{j+1} - Q_i.
    E Q[kFp ? N + 1 : 1][DL];
    S nc[kFp ? NCUR : 1];
    // complex: primed momenta k'_l and the primed column P'_{i..j} for the
    // current right end j, both built by left-to-right sums exactly as the
    // definition of P_{i,j} reads (no differences of large partial sums).
    E kp[kFp ? 1 : N][DL];
    E col[kFp ? 1 : N][DL];
    const int mu0 = s * DL;

    // ---- a1: loads; a2: sub-range momenta ----------------------------------
    if constexpr (kFp) {
#pragma unroll
      for (int c = 0; c < DL; ++c) Q[0][c] = E{};
    }
    static_for<0, N>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      E k[DL];
#pragma unroll
      for (int c = 0; c < DL; ++c) {
        k[c] = Loader<Fld>::get(a, a.momenta, l, mu0 + c, q, bad);
        J[R::idx(l, l)][c] = Loader<Fld>::get(a, a.pols, l, mu0 + c, q, bad);
      }
      k[0] = F.prime0(k[0]);
      if constexpr (kFp) {
        nc[R::idx(l, l)] = F.ndot(k, J[R::idx(l, l)]);
        k[0] = F.prime0(k[0]);
#pragma unroll
        for (int c = 0; c < DL; ++c) Q[l + 1][c] = F.eadd(Q[l][c], k[c]);
      } else {
#pragma unroll
        for (int c = 0; c < DL; ++c) kp[l][c] = k[c];
      }
    });
#pragma unroll
    for (int c = 0; c < DL; ++c) epsn[c] = Loader<Fld>::get(a, a.pols, N, mu0 + c, q, bad);

    // ---- a3/a4 (F_p): all propagator denominators, one batched inversion -----
    [[maybe_unused]] Inverses<Fld, NP> invs;
    if constexpr (kFp) {
      int32_t y[NP > 0 ? NP : 1];  // y(S) = -P_S^2
      static_for<2, N>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        static_for<0, N - m + 1>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          constexpr int j = i + m - 1;
          E Pp[DL], P[DL];
          primedP<i, j>(F, Q, Pp);
          unprime(F, Pp, P);
          y[R::pidx(i, j)] = F.ndot(Pp, P);
        });
      });
      singular = invs.compute(F, y);
    } else {
#pragma unroll
      for (int c = 0; c < DL; ++c) col[0][c] = kp[0][c];
    }

    // ---- a5: the recursion, column by column (right end j), each column from
    // the shortest range up; every range it reads is already final.
    static_for<1, N>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      if constexpr (!kFp) {
        // column j: P'_{i..j} = P'_{i..j-1} + k'_j
        static_for<0, j>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
#pragma unroll
          for (int c = 0; c < DL; ++c) col[i][c] = F.eadd(col[i][c], kp[j][c]);
        });
#pragma unroll
        for (int c = 0; c < DL; ++c) col[j][c] = kp[j][c];
      }
      static_for<0, j>([&](auto ic) {
        constexpr int i = j - 1 - decltype(ic)::value;
        constexpr bool root = (i == 0 && j == N - 1);
        E Pp[DL];
        if constexpr (kFp) {
          primedP<i, j>(F, Q, Pp);
        } else {
#pragma unroll
          for (int c = 0; c < DL; ++c) Pp[c] = col[i][c];
        }
        A K[DL];
#pragma unroll
        for (int c = 0; c < DL; ++c) K[c] = F.azero();

        // three-gluon vertex, A = [i..t], B = [t+1..j]
        S nDsum = F.szero();
        [[maybe_unused]] E PA[DL];
        static_for<i, j>([&](auto tc) {
          constexpr int t = decltype(tc)::value;
          constexpr int ia = R::idx(i, t), ib = R::idx(t + 1, j);
          const S nDm = F.ndot_u(J[ia], J[ib]);            // -(J_A.J_B)
          if constexpr (kFp) {
            // P_B.J_A = P_S.J_A - c(A),  P_A.J_B = P_S.J_B - c(B),
            // P_A - P_B = 2 Q_{t+1} - Q_i - Q_{j+1}
            const S nc2 = F.ndot_sub(Pp, J[ia], nc[ia]);   // -(P_B.J_A)
            const S nc3 = F.ndot_sub(Pp, J[ib], nc[ib]);   // -(P_A.J_B)
            F.axpy(K, F.sneg(nDm), Q[t + 1]);
            F.axpy(K, F.sneg(nc2), J[ib]);
            F.axpy(K, nc3, J[ia]);
            F.fold(K);
          } else {
#pragma unroll
            for (int c = 0; c < DL; ++c) PA[c] = (t == i) ? kp[i][c] : F.eadd(PA[c], kp[t][c]);
            const S n2 = F.ndot(col[t + 1], J[ia]);        // -(P_B.J_A)
            const S n3 = F.ndot(PA, J[ib]);                // -(P_A.J_B)
            E v[DL];
#pragma unroll
            for (int c = 0; c < DL; ++c) v[c] = F.esub(PA[c], col[t + 1][c]);
            v[0] = F.prime0(v[0]);                         // P_A - P_B
            F.axpy(K, cplx{-0.5 * nDm.re, -0.5 * nDm.im}, v);
            F.axpy(K, F.sneg(n2), J[ib]);
            F.axpy(K, n3, J[ia]);
          }
          nDsum = accumulate_scalar(F, nDsum, nDm);
        });
        const S nDhS = half_scalar(F, nDsum);
        if constexpr (kFp) {
          // -Dh(S) (Q_i + Q_{j+1})
          F.axpy(K, nDhS, Q[i]);
          F.axpy(K, nDhS, Q[j + 1]);
          F.fold(K);
        }
        if constexpr (!root) nDh[R::idx(i, j)] = nDhS;

        // four-gluon vertex: sum (J_A.J_C) J_B, then the Dh terms
        static_for<i, j - 1>([&](auto sc) {
          constexpr int s1 = decltype(sc)::value;
          static_for<s1 + 1, j>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            const S ne = F.ndot_u(J[R::idx(i, s1)], J[R::idx(t + 1, j)]);
            F.axpy(K, F.sneg(ne), J[R::idx(s1 + 1, t)]);
            constexpr int qn = v4_index<i, j>(s1, t);
            if constexpr (qn % 5 == 4) F.fold(K);
          });
        });
        F.fold(K);
        static_for<i + 1, j>([&](auto tc) {
          constexpr int t = decltype(tc)::value;
          F.axpy(K, nDh[R::idx(i, t)], J[R::idx(t + 1, j)]);
          if constexpr ((t - i) % 5 == 4) F.fold(K);
        });
        F.fold(K);
        static_for<i, j - 1>([&](auto sc) {
          constexpr int s1 = decltype(sc)::value;
          F.axpy(K, nDh[R::idx(s1 + 1, j)], J[R::idx(i, s1)]);
          if constexpr ((s1 - i) % 5 == 4) F.fold(K);
        });

        if constexpr (!root) {
          // J(S) = K' * 2/P_S^2
          S inv2;
          if constexpr (kFp) {
            inv2 = invs.get(R::pidx(i, j));
          } else {
            E P[DL];
            unprime(F, Pp, P);
            const S y = F.ndot(Pp, P);  // -P^2
            inv2 = c_inverse_times(y, -2.0, singular);
          }
          constexpr int id = R::idx(i, j);
#pragma unroll
          for (int c = 0; c < DL; ++c) J[id][c] = F.mul(F.finish(K[c]), inv2);
          if constexpr (kFp) nc[id] = F.ndot(Pp, J[id]);
        } else {
          // a6: returns -(eps_n . K'); the amplitude is M = 2 eps_n . K'
          E Kf[DL];
#pragma unroll
          for (int c = 0; c < DL; ++c) Kf[c] = F.finish(K[c]);
          result = F.ndot_u(epsn, Kf);
        }
      });
    });
  }

  __device__ static __forceinline__ void unprime(const Fld& F, const E (&Pp)[DL], E (&P)[DL]) {
#pragma unroll
    for (int c = 0; c < DL; ++c) P[c] = Pp[c];
    P[0] = F.prime0(Pp[0]);
  }

  // primed P_S = Q_{j+1} - Q_i with the time slot negated (F_p)
  template <int i, int j>
  __device__ static __forceinline__ void primedP(const Fld& F, const E (&Q)[N + 1][DL], E (&P)[DL]) {
#pragma unroll
    for (int c = 0; c < DL; ++c) P[c] = F.esub(Q[j + 1][c], Q[i][c]);
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
    const double r = f / den;
    return {y.re * r, -y.im * r};
  }
};

template <class Fld, int N, int DL, int L, int BLOCK>
__global__ __launch_bounds__(BLOCK) void bg_recursion_kernel(LaunchArgs a) {
  const int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int s = (int)(g % L);
  const int64_t q0 = g / L;
  const bool valid = q0 < a.npts;
  const int64_t q = valid ? q0 : a.npts - 1;  // tail groups recompute the last point
  uint32_t bad = 0;
  bool singular = false;
  typename Fld::S res;
  if constexpr (Fld::exact) {
    Fld F(a.fp, s);
    Recursion<Fld, N, DL, L>::run(F, a, q, s, bad, singular, res);
    if constexpr (L > 1)
      bad = group_sum<L>(bad, [](uint32_t x, uint32_t y) { return x | y; },
                         [](auto ctrl, uint32_t v) { return dpp_u32<decltype(ctrl)::value>(v); });
    if (valid && s == 0) {
      uint8_t st = bad ? PT_BADRESIDUE : (singular ? PT_SINGULAR : PT_OK);
      uint32_t outv = 0xFFFFFFFFu;
      if (st == PT_OK) {
        // res = -(eps_n . K') in Montgomery form of a value scaled by R^-4;
        // M = 2 eps_n . K' = res * (-2), times R^4 to undo the input scaling.
        int32_t m = fp_mul(res, a.fp.r4, a.fp);      // -(eps_n . K') * R^3 ... unscaled
        m = fp_sub(0, fp_add(m, m, a.fp), a.fp);     // * (-2)
        outv = fp_to_canonical(m, a.fp);
      }
      static_cast<uint32_t*>(a.out)[q] = outv;
      if (a.status) a.status[q] = st;
    }
  } else {
    Fld F(s);
    Recursion<Fld, N, DL, L>::run(F, a, q, s, bad, singular, res);
    if (valid && s == 0) {
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
