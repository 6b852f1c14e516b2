// Generic Berends-Giele recursion with a runtime number of legs (any
// 3 <= n <= 14): one point per lane, the point's current table, momenta and
// per-current scalars held in LDS as [slot][lane] columns (conflict-free,
// each lane touches its own column).  Same algebra and visiting order as
// bg_kernel.h; used for shapes without a register-resident instantiation.
#pragma once

#include "bg_kernel.h"

namespace bg {

__host__ __device__ constexpr int range_idx(int N, int i, int j) {
  return ((j - i) * (2 * N - (j - i) + 1)) / 2 + i;
}

// LDS slots per point: currents (DMAX elements each), then N + 1 vector slots
// of momenta (F_p: prefix sums Q_0..Q_N; complex: primed k'_0..k'_{N-1} and,
// in the last slot, nothing), then N column slots (complex: P'_{i..j} for the
// current right end j), then scalars nc (F_p) and nDh, then propagator
// inverses (F_p).
template <class Fld, int DMAX>
struct GenericLayout {
  using E = typename Fld::E;
  using S = typename Fld::S;
  static __host__ __device__ int ncur(int N) { return N * (N + 1) / 2 - 1; }
  static __host__ __device__ int nprop(int N) { return N * (N - 1) / 2 - 1 > 0 ? N * (N - 1) / 2 - 1 : 0; }
  static __host__ __device__ size_t bytes_per_point(int N) {
    return (size_t)(ncur(N) + 2 * N + 1) * DMAX * sizeof(E) + (size_t)2 * ncur(N) * sizeof(S) +
           (size_t)nprop(N) * sizeof(S);
  }
};

template <class Fld, int DMAX>
struct GenericRecursion {
  using E = typename Fld::E;
  using S = typename Fld::S;
  using A = typename Fld::A;
  using Lay = GenericLayout<Fld, DMAX>;
  using Rec = Recursion<Fld, 2, DMAX, 1>;  // scalar helpers
  static constexpr bool kFp = Fld::exact;

  E* Jb;   // [ncur * DMAX][P]
  E* Qb;   // [(N + 1) * DMAX][P]   F_p: Q_l; complex: k'_l
  E* Cb;   // [N * DMAX][P]         complex: column P'_{i..j}
  S* ncb;  // [ncur][P]
  S* nDb;  // [ncur][P]
  S* ivb;  // [nprop][P]
  int P, t, N;

  __device__ GenericRecursion(char* lds, int P_, int t_, int N_) : P(P_), t(t_), N(N_) {
    const int nc = Lay::ncur(N);
    Jb = reinterpret_cast<E*>(lds);
    Qb = Jb + (size_t)nc * DMAX * P;
    Cb = Qb + (size_t)(N + 1) * DMAX * P;
    ncb = reinterpret_cast<S*>(Cb + (size_t)N * DMAX * P);
    nDb = ncb + (size_t)nc * P;
    ivb = nDb + (size_t)nc * P;
  }
  __device__ __forceinline__ E& J(int r, int c) { return Jb[((size_t)r * DMAX + c) * P + t]; }
  __device__ __forceinline__ E& Q(int l, int c) { return Qb[((size_t)l * DMAX + c) * P + t]; }
  __device__ __forceinline__ E& Col(int i, int c) { return Cb[((size_t)i * DMAX + c) * P + t]; }
  __device__ __forceinline__ S& nc(int r) { return ncb[(size_t)r * P + t]; }
  __device__ __forceinline__ S& nDh(int r) { return nDb[(size_t)r * P + t]; }
  __device__ __forceinline__ S& iv(int r) { return ivb[(size_t)r * P + t]; }

  __device__ void loadJ(int r, E (&x)[DMAX]) {
#pragma unroll
    for (int c = 0; c < DMAX; ++c) x[c] = J(r, c);
  }
  __device__ void loadQ(int l, E (&x)[DMAX]) {
#pragma unroll
    for (int c = 0; c < DMAX; ++c) x[c] = Q(l, c);
  }
  __device__ void loadCol(int i, E (&x)[DMAX]) {
#pragma unroll
    for (int c = 0; c < DMAX; ++c) x[c] = Col(i, c);
  }
  __device__ void primedP(const Fld& F, int i, int j, E (&P_)[DMAX]) {
#pragma unroll
    for (int c = 0; c < DMAX; ++c) P_[c] = F.esub(Q(j + 1, c), Q(i, c));
    P_[0] = F.prime0(P_[0]);
  }

  __device__ void run(const Fld& F, const LaunchArgs& a, int64_t q, uint32_t& bad, bool& singular,
                      S& result, E (&kroot)[DMAX]) {
    const int nprop = Lay::nprop(N);
    if constexpr (kFp) {
#pragma unroll
      for (int c = 0; c < DMAX; ++c) Q(0, c) = E{};
    }
    for (int l = 0; l < N; ++l) {
      E k[DMAX], e[DMAX];
#pragma unroll
      for (int c = 0; c < DMAX; ++c) {
        k[c] = Loader<Fld>::template get<MetricRT>(a, a.momenta, l, c, q, bad);
        e[c] = Loader<Fld>::template get<MetricRT>(a, a.pols, l, c, q, bad);
        J(range_idx(N, l, l), c) = e[c];
      }
      k[0] = F.prime0(k[0]);
      if constexpr (kFp) {
        nc(range_idx(N, l, l)) = F.ndot(k, e);
        k[0] = F.prime0(k[0]);
#pragma unroll
        for (int c = 0; c < DMAX; ++c) Q(l + 1, c) = F.eadd(Q(l, c), k[c]);
      } else {
#pragma unroll
        for (int c = 0; c < DMAX; ++c) Q(l, c) = k[c];
      }
    }
    E epsn[DMAX];
#pragma unroll
    for (int c = 0; c < DMAX; ++c) epsn[c] = Loader<Fld>::template get<MetricRT>(a, a.pols, N, c, q, bad);

    // F_p propagator inverses: prefix products in iv(), y recomputed backwards
    if constexpr (kFp) {
      if (nprop > 0) {
        bool zero = false;
        int32_t acc = 0;
        for (int r = 0; r < nprop; ++r) {
          int32_t y = yprop(F, r);
          if (y == 0) { zero = true; y = F.k.one; }
          acc = (r == 0) ? y : fp_mul(acc, y, F.k);
          iv(r) = acc;
        }
        int32_t tinv = fp_pow(acc, (uint32_t)(F.k.p - 2), F.k);
        tinv = fp_mul(tinv, -F.k.two, F.k);
        for (int r = nprop - 1; r >= 0; --r) {
          int32_t y = yprop(F, r);
          if (y == 0) y = F.k.one;
          const int32_t pre = r > 0 ? iv(r - 1) : 0;
          iv(r) = r > 0 ? fp_mul(tinv, pre, F.k) : tinv;
          tinv = fp_mul(tinv, y, F.k);
        }
        singular = zero;
      }
    } else {
#pragma unroll
      for (int c = 0; c < DMAX; ++c) Col(0, c) = Q(0, c);
    }

    for (int j = 1; j < N; ++j) {
      if constexpr (!kFp) {
        for (int i = 0; i < j; ++i) {
#pragma unroll
          for (int c = 0; c < DMAX; ++c) Col(i, c) = F.eadd(Col(i, c), Q(j, c));
        }
#pragma unroll
        for (int c = 0; c < DMAX; ++c) Col(j, c) = Q(j, c);
      }
      for (int i = j - 1; i >= 0; --i) {
        const bool root = (i == 0 && j == N - 1);
        E Pp[DMAX];
        if constexpr (kFp) primedP(F, i, j, Pp);
        else loadCol(i, Pp);
        A K[DMAX];
#pragma unroll
        for (int c = 0; c < DMAX; ++c) K[c] = F.azero();
        S nDsum = F.szero();
        [[maybe_unused]] E PA[DMAX];
        for (int tt = i; tt < j; ++tt) {
          const int ia = range_idx(N, i, tt), ib = range_idx(N, tt + 1, j);
          E JA[DMAX], JB[DMAX];
          loadJ(ia, JA);
          loadJ(ib, JB);
          const S nDm = F.ndot_u(JA, JB);
          if constexpr (kFp) {
            E Qt[DMAX];
            loadQ(tt + 1, Qt);
            const S nc2 = F.ndot_sub(Pp, JA, nc(ia));
            const S nc3 = F.ndot_sub(Pp, JB, nc(ib));
            F.axpy(K, F.sneg(nDm), Qt);
            F.axpy(K, F.sneg(nc2), JB);
            F.axpy(K, nc3, JA);
            F.fold(K);
          } else {
            E kt[DMAX], PB[DMAX], v[DMAX];
            loadQ(tt, kt);
            loadCol(tt + 1, PB);
#pragma unroll
            for (int c = 0; c < DMAX; ++c) PA[c] = (tt == i) ? kt[c] : F.eadd(PA[c], kt[c]);
            const S n2 = F.ndot(PB, JA);
            const S n3 = F.ndot(PA, JB);
#pragma unroll
            for (int c = 0; c < DMAX; ++c) v[c] = F.esub(PA[c], PB[c]);
            v[0] = F.prime0(v[0]);
            F.axpy(K, cplx{-0.5 * nDm.re, -0.5 * nDm.im}, v);
            F.axpy(K, F.sneg(n2), JB);
            F.axpy(K, n3, JA);
          }
          nDsum = Rec::accumulate_scalar(F, nDsum, nDm);
        }
        const S nDhS = Rec::half_scalar(F, nDsum);
        if constexpr (kFp) {
          E Qi[DMAX], Qj[DMAX];
          loadQ(i, Qi);
          loadQ(j + 1, Qj);
          F.axpy(K, nDhS, Qi);
          F.axpy(K, nDhS, Qj);
          F.fold(K);
        }
        if (!root) nDh(range_idx(N, i, j)) = nDhS;
        int cnt = 0;
        for (int s1 = i; s1 < j - 1; ++s1) {
          E JA[DMAX];
          loadJ(range_idx(N, i, s1), JA);
          for (int tt = s1 + 1; tt < j; ++tt) {
            E JB[DMAX], JC[DMAX];
            loadJ(range_idx(N, s1 + 1, tt), JB);
            loadJ(range_idx(N, tt + 1, j), JC);
            const S ne = F.ndot_u(JA, JC);
            F.axpy(K, F.sneg(ne), JB);
            if (++cnt == 5) { F.fold(K); cnt = 0; }
          }
        }
        F.fold(K);
        cnt = 0;
        for (int tt = i + 1; tt < j; ++tt) {
          E JC[DMAX];
          loadJ(range_idx(N, tt + 1, j), JC);
          F.axpy(K, nDh(range_idx(N, i, tt)), JC);
          if (++cnt == 5) { F.fold(K); cnt = 0; }
        }
        F.fold(K);
        cnt = 0;
        for (int s1 = i; s1 < j - 1; ++s1) {
          E JA[DMAX];
          loadJ(range_idx(N, i, s1), JA);
          F.axpy(K, nDh(range_idx(N, s1 + 1, j)), JA);
          if (++cnt == 5) { F.fold(K); cnt = 0; }
        }
        if (!root) {
          S inv2;
          if constexpr (kFp) {
            inv2 = iv(range_idx(N, i, j) - N);
          } else {
            E Pu[DMAX];
#pragma unroll
            for (int c = 0; c < DMAX; ++c) Pu[c] = Pp[c];
            Pu[0] = F.prime0(Pp[0]);
            const S y = F.ndot(Pp, Pu);
            inv2 = Rec::c_inverse_times(y, -2.0, singular);
          }
          const int id = range_idx(N, i, j);
          E Jn[DMAX];
#pragma unroll
          for (int c = 0; c < DMAX; ++c) {
            Jn[c] = F.mul(F.finish(K[c]), inv2);
            J(id, c) = Jn[c];
          }
          if constexpr (kFp) nc(id) = F.ndot(Pp, Jn);
        } else {
          E Kf[DMAX];
#pragma unroll
          for (int c = 0; c < DMAX; ++c) Kf[c] = F.finish(K[c]);
          result = F.ndot_u(epsn, Kf);
#pragma unroll
          for (int c = 0; c < DMAX; ++c) kroot[c] = Kf[c];
        }
      }
    }
  }

  // -P_S^2 for propagator index r (F_p)
  __device__ int32_t yprop(const Fld& F, int r) {
    const int len = lenof(r), i = leftof(r);
    E Pp[DMAX], Pu[DMAX];
    primedP(F, i, i + len - 1, Pp);
#pragma unroll
    for (int c = 0; c < DMAX; ++c) Pu[c] = Pp[c];
    Pu[0] = F.prime0(Pp[0]);
    return F.ndot(Pp, Pu);
  }

  // propagator index r (ranges of length >= 2 in length-major order) -> length, left end
  __device__ int lenof(int r) const {
    int len = 2, base = 0;
    while (r >= base + (N - len + 1)) { base += N - len + 1; ++len; }
    return len;
  }
  __device__ int leftof(int r) const {
    int len = 2, base = 0;
    while (r >= base + (N - len + 1)) { base += N - len + 1; ++len; }
    return r - base;
  }
};

template <class Fld, int DMAX>
__global__ __launch_bounds__(256) void bg_generic_kernel(LaunchArgs a, int N) {
  extern __shared__ __align__(16) char lds[];
  const int P = blockDim.x;
  const int t = threadIdx.x;
  const int64_t q0 = (int64_t)xcd_block_index() * P + t;
  const bool valid = q0 < a.npts;
  const int64_t q = valid ? q0 : a.npts - 1;
  uint32_t bad = 0;
  bool singular = false;
  typename Fld::S res;
  typename Fld::E kroot[DMAX];
  GenericRecursion<Fld, DMAX> G(lds, P, t, N);
  if constexpr (Fld::exact) {
    Fld F(a.fp, 0);
    G.run(F, a, q, bad, singular, res, kroot);
    bad = bad >= (uint32_t)a.fp.p ? 1u : 0u;
    if (valid) {
      uint8_t st = bad ? PT_BADRESIDUE : (singular ? PT_SINGULAR : PT_OK);
      if (a.cur) {
        // root current K = 2 K', kroot scaled by R^-3: one product with R^3
#pragma unroll
        for (int c = 0; c < DMAX; ++c) {
          if (c < a.d) {
            uint32_t v = 0xFFFFFFFFu;
            if (st == PT_OK) {
              const int32_t m = fp_mul(kroot[c], a.fp.r3, a.fp);
              v = fp_to_canonical(fp_add(m, m, a.fp), a.fp);
            }
            static_cast<uint32_t*>(a.cur)[(int64_t)c * a.ld + q] = v;
          }
        }
      } else {
        uint32_t outv = 0xFFFFFFFFu;
        if (st == PT_OK) {
          int32_t m = fp_mul(res, a.fp.r4, a.fp);
          m = fp_sub(0, fp_add(m, m, a.fp), a.fp);
          outv = fp_to_canonical(m, a.fp);
        }
        static_cast<uint32_t*>(a.out)[q] = outv;
      }
      if (a.status) a.status[q] = st;
    }
  } else {
    Fld F(0);
    G.run(F, a, q, bad, singular, res, kroot);
    if (valid) {
      if (a.cur) {
#pragma unroll
        for (int c = 0; c < DMAX; ++c) {
          if (c < a.d) {
            // component 0 back from its factor i: K^0 = -i (i K^0)
            const cplx k = c == 0 ? cplx{kroot[c].im, -kroot[c].re} : kroot[c];
            double2 o;
            o.x = singular ? __builtin_nan("") : 2.0 * k.re;
            o.y = singular ? __builtin_nan("") : 2.0 * k.im;
            static_cast<double2*>(a.cur)[(int64_t)c * a.ld + q] = o;
          }
        }
      } else {
        double2 o;
        if (singular) {
          o.x = __builtin_nan("");
          o.y = __builtin_nan("");
        } else {
          o.x = -2.0 * res.re;
          o.y = -2.0 * res.im;
        }
        static_cast<double2*>(a.out)[q] = o;
      }
      if (a.status) a.status[q] = singular ? PT_SINGULAR : PT_OK;
    }
  }
}

}  // namespace bg
