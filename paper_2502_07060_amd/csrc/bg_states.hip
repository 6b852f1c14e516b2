// Polarisation states of massless d-dimensional gluons (paper Sec. 2.3), one
// point per lane: bg_states_c128 and bg_states_fp.
//
// For a massless d-vector k and a massless four-dimensional reference chi:
//   k4 = (k^0..k^3, 0, ...), mu^2 = k4.k4, c = mu^2 / (2 chi.k4),
//   kb = k4 - c chi (massless),
//   e1 = <kb|gamma|chi] / (2 [kb chi]),   e2 = [kb|gamma|chi> / <kb chi>,
//   e1~ = e2, e2~ = e1;
//   d >= 5:  e3 = kb - c chi,  e3~ = e3 / mu^2;
//   d >= 6:  e4 = (0,0,0,0, k^5, -k^4, 0..),  e4~ = e4 / mu_6^2;
//   5 <= x <= d-2:  ex^i = k^i k^{x+1} (4 <= i <= x), ex^{x+1} = -mu_{x+1}^2,
//                   ex~ = ex / (mu_{x+1}^2 mu_{x+2}^2),
// with mu_y^2 = sum_{i=4}^{y-1} (k^i)^2 (the reading of the printed d > 6
// formula in the design notes).  Spinors of a massless four-vector v use the
// chart lam = (1, (v^1 + i v^2)/v+), lamt = (v+, v^1 - i v^2) when v+ != 0
// (F_p) or |v+|^2 >= |v-|^2 (complex), else lam = ((v^1 - i v^2)/v-, 1),
// lamt = (v^1 + i v^2, v-); the four-vector of u w^T is
// ((M11+M22)/2, (M12+M21)/2, i(M12-M21)/2, (M11-M22)/2).
//
// F_p: balanced Montgomery residues (field_fp.h); i is the square root of -1
// g^((p-1)/4) for the smallest quadratic non-residue g, so p = 1 (mod 4) is
// required.  Inverses are taken in three batches (Montgomery's trick, one
// Fermat power each): the ones that need nothing else, then the spinor chart
// of kb, then the two brackets.
#include <hip/hip_runtime.h>

#include "bg.h"
#include "bg_registry.h"

namespace bg {
namespace {

constexpr int SD = BG_MAX_D;  // components held per point (d <= SD)

struct StatesArgs {
  const void* momenta;  // [d][ld]
  const void* chi;      // [4][ld]
  void* eps;            // [d-2][d][ld]
  void* epst;           // [d-2][d][ld]
  uint8_t* status;
  int64_t npts, ld;
  int d;
  FpConst fp;
  int32_t i_rep;  // F_p: Montgomery form of sqrt(-1)
  int32_t r2;     // F_p: R^2 mod p, balanced (canonical -> Montgomery form)
};

// ---- field policies ---------------------------------------------------------
struct FpOps {
  using T = int32_t;
  const FpConst& k;
  int32_t i_rep, r2;
  __device__ T add(T a, T b) const { return fp_add(a, b, k); }
  __device__ T sub(T a, T b) const { return fp_sub(a, b, k); }
  __device__ T mul(T a, T b) const { return fp_mul(a, b, k); }
  __device__ T neg(T a) const { return -a; }
  __device__ T zero() const { return 0; }
  __device__ T one() const { return k.one; }
  __device__ T half() const { return k.inv2; }
  __device__ T two() const { return k.two; }
  __device__ T iu() const { return i_rep; }
  __device__ bool is_zero(T a) const { return a == 0; }
  __device__ bool plus_chart(T vp, T) const { return vp != 0; }
  // x_s <- 1 / x_s for s < n (all non-zero), one Fermat power
  template <int M>
  __device__ void inv_batch(T (&x)[M], int n) const {
    T pre[M];
    T acc = k.one;
#pragma unroll
    for (int s = 0; s < M; ++s)
      if (s < n) {
        acc = fp_mul(acc, x[s], k);
        pre[s] = acc;
      }
    T t = fp_pow(acc, (uint32_t)(k.p - 2), k);
#pragma unroll
    for (int s = M - 1; s >= 0; --s)
      if (s < n) {
        const T xs = x[s];
        x[s] = s > 0 ? fp_mul(t, pre[s - 1], k) : t;
        t = fp_mul(t, xs, k);
      }
  }
};

struct COps {
  using T = cplx;
  __device__ T add(T a, T b) const { return cadd(a, b); }
  __device__ T sub(T a, T b) const { return csub(a, b); }
  __device__ T mul(T a, T b) const { return cmul(a, b); }
  __device__ T neg(T a) const { return cneg(a); }
  __device__ T zero() const { return {0.0, 0.0}; }
  __device__ T one() const { return {1.0, 0.0}; }
  __device__ T half() const { return {0.5, 0.0}; }
  __device__ T two() const { return {2.0, 0.0}; }
  __device__ T iu() const { return {0.0, 1.0}; }
  __device__ bool is_zero(T a) const { return a.re == 0.0 && a.im == 0.0; }
  __device__ bool plus_chart(T vp, T vm) const {
    return vp.re * vp.re + vp.im * vp.im >= vm.re * vm.re + vm.im * vm.im;
  }
  template <int M>
  __device__ void inv_batch(T (&x)[M], int n) const {
#pragma unroll
    for (int s = 0; s < M; ++s)
      if (s < n) {
        const double den = x[s].re * x[s].re + x[s].im * x[s].im;
        x[s] = {x[s].re / den, -x[s].im / den};
      }
  }
};

template <class Ops, class T>
__device__ __forceinline__ T mdot4(const Ops& o, const T* x, const T* y) {
  T s = o.mul(x[0], y[0]);
#pragma unroll
  for (int m = 1; m < 4; ++m) s = o.sub(s, o.mul(x[m], y[m]));
  return s;
}

// the four-vector of u w^T
template <class Ops, class T>
__device__ __forceinline__ void vec_of(const Ops& o, const T* u, const T* w, T* out) {
  const T m11 = o.mul(u[0], w[0]), m12 = o.mul(u[0], w[1]);
  const T m21 = o.mul(u[1], w[0]), m22 = o.mul(u[1], w[1]);
  out[0] = o.mul(o.add(m11, m22), o.half());
  out[1] = o.mul(o.add(m12, m21), o.half());
  out[2] = o.mul(o.mul(o.iu(), o.sub(m12, m21)), o.half());
  out[3] = o.mul(o.sub(m11, m22), o.half());
}

// spinors of a massless four-vector given the inverse of its chart component
template <class Ops, class T>
__device__ __forceinline__ void spinors(const Ops& o, const T* v, bool plus, T inv_chart, T* lam, T* lamt) {
  const T vp = o.add(v[0], v[3]), vm = o.sub(v[0], v[3]);
  const T iv2 = o.mul(o.iu(), v[2]);
  const T vt = o.add(v[1], iv2), vtb = o.sub(v[1], iv2);
  if (plus) {
    lam[0] = o.one();
    lam[1] = o.mul(vt, inv_chart);
    lamt[0] = vp;
    lamt[1] = vtb;
  } else {
    lam[0] = o.mul(vtb, inv_chart);
    lam[1] = o.one();
    lamt[0] = vt;
    lamt[1] = vm;
  }
}

template <class Ops, class T>
__device__ __forceinline__ T bracket(const Ops& o, const T* a, const T* b) {
  return o.sub(o.mul(a[0], b[1]), o.mul(a[1], b[0]));
}

// sum_{i=4}^{y-1} (k^i)^2
template <class Ops, class T>
__device__ __forceinline__ T mu2y(const Ops& o, const T* k, int y) {
  T s = o.zero();
#pragma unroll
  for (int i = 4; i < SD; ++i)
    if (i < y) s = o.add(s, o.mul(k[i], k[i]));
  return s;
}

// all d - 2 states and their duals of one point, handed to emit(state,
// component, e, e~) in order (every component, zeros included); false (and
// nothing emitted) if a required denominator vanishes
template <class Ops, class T, class Emit>
__device__ bool point_states(const Ops& o, const T* k, const T* chi, int d, Emit&& emit) {
  T k4[4], ch[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    k4[m] = k[m];
    ch[m] = chi[m];
  }
  const T mu2 = mdot4(o, k4, k4);
  const T ck = mdot4(o, ch, k4);
  // batch 1: 2 chi.k4, the chart component of chi, mu^2 (d >= 5), mu_6^2
  // (d >= 6), mu_{x+1}^2 mu_{x+2}^2 (5 <= x <= d-2)
  const T vpc = o.add(ch[0], ch[3]), vmc = o.sub(ch[0], ch[3]);
  const bool plus_c = o.plus_chart(vpc, vmc);
  // fixed slots (unused ones hold 1): 0 2 chi.k4, 1 chi chart, 2 mu^2,
  // 3 mu_6^2, 4 + (x - 5) the product for the extra state x
  constexpr int NB1 = 4 + (SD - 6);
  T b1[NB1];
  b1[0] = o.add(ck, ck);
  b1[1] = plus_c ? vpc : vmc;
  b1[2] = d >= 5 ? mu2 : o.one();
  b1[3] = d >= 6 ? mu2y(o, k, 6) : o.one();
#pragma unroll
  for (int x = 5; x < SD - 1; ++x)
    b1[4 + x - 5] = x <= d - 2 ? o.mul(mu2y(o, k, x + 1), mu2y(o, k, x + 2)) : o.one();
  bool sing = false;
#pragma unroll
  for (int s = 0; s < NB1; ++s)
    if (o.is_zero(b1[s])) {
      sing = true;
      b1[s] = o.one();
    }
  o.inv_batch(b1, NB1);
  const T c = o.mul(mu2, b1[0]);
  T kb[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) kb[m] = o.sub(k4[m], o.mul(c, ch[m]));
  T lc[2], tc[2];
  spinors(o, ch, plus_c, b1[1], lc, tc);
  // batch 2: the chart component of kb
  const T vpk = o.add(kb[0], kb[3]), vmk = o.sub(kb[0], kb[3]);
  const bool plus_k = o.plus_chart(vpk, vmk);
  T b2[1] = {plus_k ? vpk : vmk};
  if (o.is_zero(b2[0])) {
    sing = true;
    b2[0] = o.one();
  }
  o.inv_batch(b2, 1);
  T lk[2], tk[2];
  spinors(o, kb, plus_k, b2[0], lk, tk);
  // batch 3: [kb chi], <kb chi>
  T b3[2] = {bracket(o, tk, tc), bracket(o, lk, lc)};
#pragma unroll
  for (int s = 0; s < 2; ++s)
    if (o.is_zero(b3[s])) {
      sing = true;
      b3[s] = o.one();
    }
  o.inv_batch(b3, 2);
  if (sing) return false;

  const T z = o.zero();
  T e1[4], e2[4], v[4];
  vec_of(o, lk, tc, v);
#pragma unroll
  for (int m = 0; m < 4; ++m) e1[m] = o.mul(v[m], b3[0]);
  vec_of(o, lc, tk, v);
  const T two_over_an = o.mul(o.two(), b3[1]);
#pragma unroll
  for (int m = 0; m < 4; ++m) e2[m] = o.mul(v[m], two_over_an);
#pragma unroll
  for (int m = 0; m < SD; ++m)
    if (m < d) {
      emit(0, m, m < 4 ? e1[m] : z, m < 4 ? e2[m] : z);
      emit(1, m, m < 4 ? e2[m] : z, m < 4 ? e1[m] : z);
    }
  if (d >= 5) {
#pragma unroll
    for (int m = 0; m < SD; ++m)
      if (m < d) {
        const T e3 = m < 4 ? o.sub(kb[m], o.mul(c, ch[m])) : z;
        emit(2, m, e3, o.mul(e3, b1[2]));
      }
  }
  if (d >= 6) {
#pragma unroll
    for (int m = 0; m < SD; ++m)
      if (m < d) {
        const T e4 = m == 4 ? k[5] : (m == 5 ? o.neg(k[4]) : z);
        emit(3, m, e4, o.mul(e4, b1[3]));
      }
  }
#pragma unroll
  for (int x = 5; x < SD - 1; ++x) {
    if (x <= d - 2) {
      const T kx1 = k[x + 1];
      const T top = o.neg(mu2y(o, k, x + 1));
#pragma unroll
      for (int m = 0; m < SD; ++m)
        if (m < d) {
          const T ex = (m >= 4 && m <= x) ? o.mul(k[m], kx1) : (m == x + 1 ? top : z);
          emit(x - 1, m, ex, o.mul(ex, b1[4 + x - 5]));  // e_x is state number x, slot x - 1
        }
    }
  }
  return true;
}

__global__ __launch_bounds__(256) void states_fp_kernel(StatesArgs a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.npts) return;
  const FpOps o{a.fp, a.i_rep, a.r2};
  const uint32_t* km = static_cast<const uint32_t*>(a.momenta);
  const uint32_t* cm = static_cast<const uint32_t*>(a.chi);
  int32_t k[SD], chi[4];
  bool bad = false;
#pragma unroll
  for (int m = 0; m < SD; ++m) {
    k[m] = 0;
    if (m < a.d) {
      const uint32_t x = km[(int64_t)m * a.ld + q];
      bad |= x >= (uint32_t)a.fp.p;
      k[m] = fp_mul(fp_from_canonical(x < (uint32_t)a.fp.p ? x : 0u, a.fp), a.r2, a.fp);
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const uint32_t x = cm[(int64_t)m * a.ld + q];
    bad |= x >= (uint32_t)a.fp.p;
    chi[m] = fp_mul(fp_from_canonical(x < (uint32_t)a.fp.p ? x : 0u, a.fp), a.r2, a.fp);
  }
  uint32_t* eo = static_cast<uint32_t*>(a.eps);
  uint32_t* to = static_cast<uint32_t*>(a.epst);
  const auto emit = [&](int s, int m, int32_t e, int32_t et) {
    const int64_t off = ((int64_t)s * a.d + m) * a.ld + q;
    eo[off] = fp_to_canonical(fp_mul(e, 1, a.fp), a.fp);   // Montgomery form -> residue
    to[off] = fp_to_canonical(fp_mul(et, 1, a.fp), a.fp);
  };
  const bool ok = !bad && point_states(o, k, chi, a.d, emit);
  if (!ok) {
    for (int s = 0; s < a.d - 2; ++s)
      for (int m = 0; m < a.d; ++m) {
        const int64_t off = ((int64_t)s * a.d + m) * a.ld + q;
        eo[off] = 0xFFFFFFFFu;
        to[off] = 0xFFFFFFFFu;
      }
  }
  if (a.status) a.status[q] = bad ? PT_BADRESIDUE : (ok ? PT_OK : PT_SINGULAR);
}

__global__ __launch_bounds__(256) void states_c128_kernel(StatesArgs a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.npts) return;
  const COps o{};
  const double2* km = static_cast<const double2*>(a.momenta);
  const double2* cm = static_cast<const double2*>(a.chi);
  cplx k[SD], chi[4];
#pragma unroll
  for (int m = 0; m < SD; ++m) {
    k[m] = {0.0, 0.0};
    if (m < a.d) {
      const double2 x = km[(int64_t)m * a.ld + q];
      k[m] = {x.x, x.y};
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const double2 x = cm[(int64_t)m * a.ld + q];
    chi[m] = {x.x, x.y};
  }
  double2* eo = static_cast<double2*>(a.eps);
  double2* to = static_cast<double2*>(a.epst);
  const auto emit = [&](int s, int m, cplx e, cplx et) {
    const int64_t off = ((int64_t)s * a.d + m) * a.ld + q;
    eo[off] = double2{e.re, e.im};
    to[off] = double2{et.re, et.im};
  };
  const bool ok = point_states(o, k, chi, a.d, emit);
  if (!ok) {
    const double nan = __builtin_nan("");
    for (int s = 0; s < a.d - 2; ++s)
      for (int m = 0; m < a.d; ++m) {
        const int64_t off = ((int64_t)s * a.d + m) * a.ld + q;
        eo[off] = double2{nan, nan};
        to[off] = double2{nan, nan};
      }
  }
  if (a.status) a.status[q] = ok ? PT_OK : PT_SINGULAR;
}

int64_t mulmod(int64_t a, int64_t b, int64_t p) { return (int64_t)((__int128)a * b % p); }

int64_t powmod64(int64_t a, int64_t e, int64_t p) {
  int64_t r = 1 % p;
  a %= p;
  while (e) {
    if (e & 1) r = mulmod(r, a, p);
    a = mulmod(a, a, p);
    e >>= 1;
  }
  return r;
}

int32_t balanced32(int64_t x, int64_t p) {
  x %= p;
  if (x < 0) x += p;
  return x > (p - 1) / 2 ? (int32_t)(x - p) : (int32_t)x;
}

int launch_states(bool fp, int d, int64_t npts, int64_t ld, uint32_t p, const void* momenta, const void* chi,
                  void* eps, void* epst, uint8_t* status, void* stream) {
  if (d < 4 || d > BG_MAX_D) return BG_EDOMAIN;
  if (npts < 0) return BG_EINVAL;
  if (fp && (p < 3 || p >= 0x80000000u || !is_prime_u32(p))) return BG_ENOTPRIME;
  if (fp && p % 4 != 1) return BG_EDOMAIN;  // no square root of -1 in F_p
  if (npts == 0) return BG_OK;
  if (ld < npts || !momenta || !chi || !eps || !epst) return BG_EINVAL;
  StatesArgs a{};
  a.momenta = momenta;
  a.chi = chi;
  a.eps = eps;
  a.epst = epst;
  a.status = status;
  a.npts = npts;
  a.ld = ld;
  a.d = d;
  if (fp) {
    a.fp = make_fp_const(p);
    const int64_t R = powmod64(2, 64, p);
    a.i_rep = fp_sqrt_minus_one_mont(p);
    a.r2 = balanced32(mulmod(R, R, p), p);
  }
  const int64_t blocks = (npts + 255) / 256;
  if (blocks > 0x7FFFFFFF) return BG_EINVAL;
  void* args[] = {&a};
  const hipError_t e = hipLaunchKernel(fp ? reinterpret_cast<const void*>(&states_fp_kernel)
                                          : reinterpret_cast<const void*>(&states_c128_kernel),
                                       dim3((unsigned)blocks), dim3(256), args, 0, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BG_OK : BG_EHIP;
}

// ---------------------------------------------------------------------------
// sums over the states of one cut leg: S = sum_s (e_s . K_L)(e~_s . K_R)
// ---------------------------------------------------------------------------
// With K_L, K_R the root currents of two trees whose last leg is the cut leg
// (momentum l in one, -l in the other), M_L(e_s) = e_s . K_L and
// M_R(e~_s) = e~_s . K_R, so S is the state sum of their product (paper
// Sec. 2.1, the leading pole of the cut equation; Sec. 2.3 states).  One
// point per lane; mostly-minus products.
struct StateSumArgs {
  const void* kl;
  const void* kr;
  const void* eps;
  const void* epst;
  void* out;
  uint8_t* status;
  int64_t npts, ld;
  int d;
  FpConst fp;
};

__global__ __launch_bounds__(256) void state_sum_fp_kernel(StateSumArgs a) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= a.npts) return;
  const FpConst& F = a.fp;
  const uint32_t* kl = static_cast<const uint32_t*>(a.kl);
  const uint32_t* kr = static_cast<const uint32_t*>(a.kr);
  const uint32_t* ep = static_cast<const uint32_t*>(a.eps);
  const uint32_t* et = static_cast<const uint32_t*>(a.epst);
  uint32_t maxraw = 0;
  auto rd = [&](const uint32_t* base, int64_t e) {
    const uint32_t v = base[e * a.ld + q];
    maxraw = maxraw > v ? maxraw : v;
    return fp_from_canonical(v < (uint32_t)F.p ? v : 0u, F);
  };
  int32_t L[BG_MAX_D], Rv[BG_MAX_D];
#pragma unroll
  for (int mu = 0; mu < BG_MAX_D; ++mu) {
    L[mu] = mu < a.d ? rd(kl, mu) : 0;
    Rv[mu] = mu < a.d ? rd(kr, mu) : 0;
  }
  L[0] = -L[0];  // primed: sum_mu L'_mu x_mu = -(L . x)
  Rv[0] = -Rv[0];
  // (e.K_L)(e~.K_R) = (-(e.K_L))(-(e~.K_R)); each dot is an int64 sum of
  // balanced products (a fold after every four), reduced to t R^-1; the
  // products of two such are summed in int64 and reduced once more (R^-3),
  // and one product with R^4 restores S
  int64_t acc = 0;
  for (int s = 0; s < a.d - 2; ++s) {
    int64_t tl = 0, tr = 0;
#pragma unroll
    for (int mu = 0; mu < BG_MAX_D; ++mu) {
      if (mu < a.d) {
        tl = mad64(rd(ep, (int64_t)s * a.d + mu), L[mu], tl);
        tr = mad64(rd(et, (int64_t)s * a.d + mu), Rv[mu], tr);
      }
      if ((mu & 3) == 3) {
        tl = fp_fold(tl, F);
        tr = fp_fold(tr, F);
      }
    }
    const int32_t dl = fp_redc2(fp_fold(tl, F), F), dr = fp_redc2(fp_fold(tr, F), F);
    acc = fp_fold(mad64(dl, dr, acc), F);
  }
  const bool bad = maxraw >= (uint32_t)F.p;
  const int32_t sum = fp_mul(fp_redc2(acc, F), F.r4, F);
  static_cast<uint32_t*>(a.out)[q] = bad ? 0xFFFFFFFFu : fp_to_canonical(sum, F);
  if (a.status) a.status[q] = bad ? PT_BADRESIDUE : PT_OK;
}

__global__ __launch_bounds__(256) void state_sum_c128_kernel(StateSumArgs a) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= a.npts) return;
  const double2* kl = static_cast<const double2*>(a.kl);
  const double2* kr = static_cast<const double2*>(a.kr);
  const double2* ep = static_cast<const double2*>(a.eps);
  const double2* et = static_cast<const double2*>(a.epst);
  double2 L[BG_MAX_D], Rv[BG_MAX_D];
  bool nan = false;
#pragma unroll
  for (int mu = 0; mu < BG_MAX_D; ++mu) {
    L[mu] = mu < a.d ? kl[(int64_t)mu * a.ld + q] : double2{0.0, 0.0};
    Rv[mu] = mu < a.d ? kr[(int64_t)mu * a.ld + q] : double2{0.0, 0.0};
  }
  double sre = 0.0, sim = 0.0;
  for (int s = 0; s < a.d - 2; ++s) {
    double lre = 0.0, lim = 0.0, rre = 0.0, rim = 0.0;
#pragma unroll
    for (int mu = 0; mu < BG_MAX_D; ++mu) {
      if (mu < a.d) {
        const double g = mu == 0 ? 1.0 : -1.0;
        const double2 e = ep[((int64_t)s * a.d + mu) * a.ld + q];
        const double2 f = et[((int64_t)s * a.d + mu) * a.ld + q];
        lre = __builtin_fma(g * e.x, L[mu].x, __builtin_fma(-g * e.y, L[mu].y, lre));
        lim = __builtin_fma(g * e.x, L[mu].y, __builtin_fma(g * e.y, L[mu].x, lim));
        rre = __builtin_fma(g * f.x, Rv[mu].x, __builtin_fma(-g * f.y, Rv[mu].y, rre));
        rim = __builtin_fma(g * f.x, Rv[mu].y, __builtin_fma(g * f.y, Rv[mu].x, rim));
      }
    }
    sre = __builtin_fma(lre, rre, __builtin_fma(-lim, rim, sre));
    sim = __builtin_fma(lre, rim, __builtin_fma(lim, rre, sim));
  }
  nan = sre != sre || sim != sim;
  static_cast<double2*>(a.out)[q] = double2{sre, sim};
  if (a.status) a.status[q] = nan ? PT_SINGULAR : PT_OK;
}

int launch_state_sum(bool fp, int d, int64_t npts, int64_t ld, uint32_t p, const void* kl, const void* kr,
                     const void* eps, const void* epst, void* out, uint8_t* status, void* stream) {
  if (d < 4 || d > BG_MAX_D) return BG_EDOMAIN;
  if (fp && (p < 3 || p >= 0x80000000u || !is_prime_u32(p))) return BG_ENOTPRIME;
  if (npts < 0) return BG_EINVAL;
  if (npts == 0) return BG_OK;
  if (ld < npts || !kl || !kr || !eps || !epst || !out) return BG_EINVAL;
  StateSumArgs a{};
  a.kl = kl;
  a.kr = kr;
  a.eps = eps;
  a.epst = epst;
  a.out = out;
  a.status = status;
  a.npts = npts;
  a.ld = ld;
  a.d = d;
  if (fp) a.fp = make_fp_const(p);
  const int64_t blocks = (npts + 255) / 256;
  if (blocks > 0x7FFFFFFF) return BG_EINVAL;
  void* args[] = {&a};
  const hipError_t e = hipLaunchKernel(fp ? reinterpret_cast<const void*>(&state_sum_fp_kernel)
                                          : reinterpret_cast<const void*>(&state_sum_c128_kernel),
                                       dim3((unsigned)blocks), dim3(256), args, 0, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BG_OK : BG_EHIP;
}

}  // namespace
}  // namespace bg

extern "C" {

int bg_state_sum_c128(int d, int64_t npts, int64_t ld, const double* kl, const double* kr, const double* eps,
                      const double* epst, double* out, uint8_t* status, void* hip_stream) {
  return bg::launch_state_sum(false, d, npts, ld, 0, kl, kr, eps, epst, out, status, hip_stream);
}

int bg_state_sum_fp(int d, int64_t npts, int64_t ld, uint32_t p, const uint32_t* kl, const uint32_t* kr,
                    const uint32_t* eps, const uint32_t* epst, uint32_t* out, uint8_t* status, void* hip_stream) {
  return bg::launch_state_sum(true, d, npts, ld, p, kl, kr, eps, epst, out, status, hip_stream);
}

int bg_states_c128(int d, int64_t npts, int64_t ld, const double* momenta, const double* chi, double* eps,
                   double* epst, uint8_t* status, void* hip_stream) {
  return bg::launch_states(false, d, npts, ld, 0, momenta, chi, eps, epst, status, hip_stream);
}

int bg_states_fp(int d, int64_t npts, int64_t ld, uint32_t p, const uint32_t* momenta, const uint32_t* chi,
                 uint32_t* eps, uint32_t* epst, uint8_t* status, void* hip_stream) {
  return bg::launch_states(true, d, npts, ld, p, momenta, chi, eps, epst, status, hip_stream);
}

}  // extern "C"
