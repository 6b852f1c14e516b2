// From F_p samples back to rational numbers (paper Sec. 1 and Sec. 3: the
// finite-field values at rational kinematic points are reconstructed as
// rationals, as in the comparison with Caravel):
//
//   bg_fp_from_rational      residues n/d mod p of int64 fractions, for
//                            feeding rational kinematics to bg_amplitudes_fp;
//   bg_rational_reconstruct  Chinese remaindering of one residue per prime
//                            followed by rational reconstruction, one point
//                            per lane.
//
// Reconstruction (Wang; von zur Gathen and Gerhard, Modern Computer Algebra,
// Sec. 5.10).  With M = p_1 ... p_k and B = floor(sqrt((M - 1) / 2)):
// the residues give 0 <= x < M (Garner's mixed-radix form, then Horner in
// 32-bit limbs); the extended Euclidean algorithm runs on r_0 = M, r_1 = x,
// t_0 = 0, t_1 = 1 (every r_j = s_j M + t_j x) until the first r_j <= B; the
// result is sign(t_j) r_j / |t_j| when 0 < |t_j| <= B and gcd(t_j, M) = 1
// (which equals gcd(r_j, t_j) = 1, since gcd(s_j, t_j) = 1), else there is
// none.  A fraction with |a| <= B, 0 < b <= B, gcd(a, b) = 1 and a = b x
// (mod M) is unique (2 B^2 < M) and is what this returns.
//
// Limb arithmetic.  Numbers are K 32-bit limbs (K >= number of primes, so
// M < 2^(31 K)); the Euclidean cofactors t_j are kept in two's complement
// modulo 2^(32 K), which is exact because |t_j| <= M < 2^(32 K - 1).  Every
// limb loop is unrolled over K (no run-time register indexing).  A quotient
// is estimated from the two remainders converted to binary64 (M < 2^992 is
// within range, relative error below 2^-52): below 2^31 it is taken whole and
// corrected by at most a few units; larger quotients are removed in pieces of
// 64 bits aligned to a limb, each an under-estimate, so a remainder never
// goes negative there.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <vector>

#include "bg.h"
#include "bg_registry.h"
#include "field_fp.h"

namespace bg {
namespace {

// ---------------------------------------------------------------------------
// residues of fractions
// ---------------------------------------------------------------------------
constexpr int kResidueChunk = 16;  // values per lane: one Fermat power per chunk

struct ResidueArgs {
  const int64_t* num;
  const int64_t* den;
  uint32_t* out;
  uint8_t* status;
  int64_t count;
  FpConst fp;
  int32_t r3;  // R^3 mod p: x R^-1 -> x R
};

// x (any int64) -> x R mod p, balanced (Montgomery form)
__device__ __forceinline__ int32_t mont_of_i64(int64_t x, const FpConst& F, int32_t r3) {
  return fp_mul(fp_redc2(fp_fold(x, F), F), r3, F);
}

__global__ __launch_bounds__(256) void residue_kernel(ResidueArgs a) {
  const int64_t base = ((int64_t)blockIdx.x * 256 + threadIdx.x) * kResidueChunk;
  if (base >= a.count) return;
  const FpConst& F = a.fp;
  const int cnt = (int)(a.count - base < kResidueChunk ? a.count - base : kResidueChunk);
  int32_t nm[kResidueChunk], dm[kResidueChunk];
  bool zero[kResidueChunk];
  int32_t acc = F.one;
  // Montgomery batch inversion of the denominators (Montgomery 1987); a zero
  // denominator is replaced by 1 and its value flagged.  Forward: acc =
  // d_0 ... d_u, and n_u is multiplied by d_0 ... d_{u-1}.
#pragma unroll
  for (int u = 0; u < kResidueChunk; ++u) {
    if (u < cnt) {
      nm[u] = mont_of_i64(a.num[base + u], F, a.r3);
      dm[u] = mont_of_i64(a.den[base + u], F, a.r3);
      zero[u] = dm[u] == 0;
      if (zero[u]) dm[u] = F.one;
      nm[u] = fp_mul(nm[u], acc, F);
      acc = fp_mul(acc, dm[u], F);
    }
  }
  int32_t inv = fp_pow(acc, (uint32_t)(F.p - 2), F);  // 1 / (d_0 ... d_{cnt-1})
  // backward: inv = 1 / (d_0 ... d_u), so n_u (d_0 ... d_{u-1}) inv = n_u / d_u
#pragma unroll
  for (int u = kResidueChunk - 1; u >= 0; --u) {
    if (u < cnt) {
      const int32_t q = fp_mul(nm[u], inv, F);
      inv = fp_mul(inv, dm[u], F);
      const int32_t v = fp_redc2((int64_t)q, F);  // out of Montgomery form, balanced
      a.out[base + u] = zero[u] ? 0xFFFFFFFFu : fp_to_canonical(v, F);
      if (a.status) a.status[base + u] = zero[u] ? 1 : 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Chinese remaindering and rational reconstruction
// ---------------------------------------------------------------------------
struct PrimeConst {
  int32_t p, h, c32, c64, r2, minv;  // minv = (p_0 ... p_{i-1})^-1 R mod p_i
  uint32_t pinv;
};

struct RRArgs {
  const uint32_t* residues;  // [nprimes][ld]
  int32_t* num;              // [L][ld] two's complement limbs
  uint32_t* den;             // [L][ld]
  uint8_t* status;
  int64_t npts, ld;
  int nprimes, L;
  PrimeConst pc[BG_RR_MAX_PRIMES];
  uint32_t M[BG_RR_MAX_PRIMES];
  uint32_t B[BG_RR_MAX_PRIMES];
};

__device__ __forceinline__ FpConst fpc(const PrimeConst& c) {
  FpConst F{};
  F.p = c.p;
  F.h = c.h;
  F.pinv = c.pinv;
  F.negp = -c.p;
  F.c32 = c.c32;
  F.c64 = c.c64;
  F.one = c.c64;
  return F;
}

// x < 2^31 -> x R mod p (Montgomery form, balanced)
__device__ __forceinline__ int32_t mont_small(int32_t x, const FpConst& F, int32_t r2) {
  return fp_mul(fp_norm(x, F), r2, F);
}

template <int K>
__device__ __forceinline__ int cmp(const uint32_t (&x)[K], const uint32_t (&y)[K]) {
  int c = 0;
#pragma unroll
  for (int k = K - 1; k >= 0; --k)
    if (c == 0) c = (x[k] > y[k]) - (x[k] < y[k]);
  return c;
}

template <int K>
__device__ __forceinline__ double to_double(const uint32_t (&x)[K]) {
  double v = 0.0;
#pragma unroll
  for (int k = K - 1; k >= 0; --k) v = v * 4294967296.0 + (double)x[k];
  return v;
}

// x -= c y (mod 2^(32K)); returns the borrow out of the top limb as a signed
// count (negative iff x < c y when both are read as unsigned)
template <int K>
__device__ __forceinline__ int64_t submul(uint32_t (&x)[K], const uint32_t (&y)[K], uint32_t c) {
  uint64_t carry = 0;
  int64_t borrow = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t prod = (uint64_t)c * y[k] + carry;
    carry = prod >> 32;
    const int64_t diff = (int64_t)x[k] - (int64_t)(uint32_t)prod + borrow;
    x[k] = (uint32_t)diff;
    borrow = diff >> 32;
  }
  return borrow - (int64_t)carry;
}

template <int K>
__device__ __forceinline__ void sub_from(uint32_t (&x)[K], const uint32_t (&y)[K]) {
  int64_t borrow = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t d = (int64_t)x[k] - (int64_t)y[k] + borrow;
    x[k] = (uint32_t)d;
    borrow = d >> 32;
  }
}

// y << 32 s (limbs), s in [0, K): a barrel shifter of static moves
template <int K>
__device__ __forceinline__ void shift_limbs(const uint32_t (&y)[K], int s, uint32_t (&out)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = y[k];
#pragma unroll
  for (int b = 1; b < K; b <<= 1) {
    const bool on = (s & b) != 0;
#pragma unroll
    for (int k = K - 1; k >= 0; --k) out[k] = on ? (k >= b ? out[k - b] : 0u) : out[k];
  }
}

template <int K>
__device__ __forceinline__ void negate(uint32_t (&x)[K]) {
  uint64_t carry = 1;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t s = (uint64_t)(~x[k]) + carry;
    x[k] = (uint32_t)s;
    carry = s >> 32;
  }
}

template <int K>
__device__ __forceinline__ bool is_zero(const uint32_t (&x)[K]) {
  uint32_t o = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) o |= x[k];
  return o == 0;
}

// |x| mod p for x < 2^(32K): sum of limb_k 2^(32k) R, folded, then one REDC
template <int K>
__device__ __forceinline__ int32_t mod_prime(const uint32_t (&x)[K], const FpConst& F, int32_t c32m) {
  int64_t T = 0;
  int32_t w = F.one;  // 2^(32k) R mod p
#pragma unroll
  for (int k = 0; k < K; ++k) {
    T = fp_fold(T + (int64_t)x[k] * (int64_t)w, F);
    w = fp_mul(w, c32m, F);
  }
  return fp_redc2(T, F);
}

template <int K>
__global__ __launch_bounds__(256) void rr_kernel(RRArgs a) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= a.npts) return;
  const int P = a.nprimes;
  uint8_t st = 0;
  // ---- residues and Garner's mixed-radix digits v_i (x = v_0 + p_0 (v_1 + p_1 (...)))
  uint32_t v[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    v[i] = 0;
    if (i < P) {
      const FpConst F = fpc(a.pc[i]);
      const uint32_t r = a.residues[(int64_t)i * a.ld + q];
      if (r >= (uint32_t)F.p) st = 2;
      // X_{i-1} mod p_i by Horner over the digits found so far
      int32_t t = 0;
#pragma unroll
      for (int j = i - 1; j >= 0; --j) {
        const int32_t pj = mont_small(a.pc[j].p, F, a.pc[i].r2);
        t = fp_add(fp_mul(t, pj, F), mont_small((int32_t)v[j], F, a.pc[i].r2), F);
      }
      const int32_t rm = mont_small((int32_t)(r < (uint32_t)F.p ? r : 0u), F, a.pc[i].r2);
      const int32_t d = fp_mul(fp_sub(rm, t, F), a.pc[i].minv, F);  // Montgomery form of v_i
      v[i] = fp_to_canonical(fp_redc2((int64_t)d, F), F);
    }
  }
  // ---- x = v_{P-1}; x = x p_i + v_i for i = P-2 .. 0
  uint32_t x[K];
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] = 0;
#pragma unroll
  for (int i = K - 1; i >= 0; --i) {
    if (i < P) {
      uint64_t carry = v[i];
      const uint32_t p = (uint32_t)a.pc[i].p;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint64_t s = (uint64_t)x[k] * p + carry;
        x[k] = (uint32_t)s;
        carry = s >> 32;
      }
    }
  }
  // ---- extended Euclid on (M, x) until the remainder is <= B
  uint32_t r0[K], r1[K], t0[K], t1[K], Bv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    r0[k] = a.M[k];
    r1[k] = x[k];
    t0[k] = 0;
    t1[k] = k == 0 ? 1u : 0u;
    Bv[k] = a.B[k];
  }
  // every step shrinks the remainders: a small quotient step at least halves
  // r_j two steps on, a large-quotient piece removes 32 bits or more; the cap
  // only guarantees that every lane leaves the loop
  const int cap = 96 * K + 64;
  int it = 0;
  while (cmp(r1, Bv) > 0 && it < cap) {
    ++it;
    const double qe = to_double(r0) / to_double(r1);
    if (qe < 2147483648.0) {
      uint32_t qq = (uint32_t)qe;
      int64_t bo = submul(r0, r1, qq);
      while (bo < 0) {  // over-estimate: add r1 back
        uint64_t carry = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const uint64_t s = (uint64_t)r0[k] + r1[k] + carry;
          r0[k] = (uint32_t)s;
          carry = s >> 32;
        }
        bo += (int64_t)carry;
        --qq;
      }
      while (cmp(r0, r1) >= 0) {  // under-estimate
        sub_from(r0, r1);
        ++qq;
      }
      (void)submul(t0, t1, qq);
      // (r0, r1) <- (r1, r0 - q r1), (t0, t1) <- (t1, t0 - q t1)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t a0 = r0[k];
        r0[k] = r1[k];
        r1[k] = a0;
        const uint32_t b0 = t0[k];
        t0[k] = t1[k];
        t1[k] = b0;
      }
    } else {
      // take c 2^(32 s) out of the quotient, c < 2^64 an under-estimate
      int e = 0;
      (void)frexp(qe, &e);  // qe in [2^(e-1), 2^e)
      const int s = e > 64 ? (e - 64 + 31) / 32 : 0;
      const double scaled = ldexp(qe, -32 * s) * (1.0 - 0x1p-40);
      uint64_t c = scaled >= 18446744073709551616.0 ? ~0ull : (uint64_t)scaled;
      if (c > 0) c -= 1;
      uint32_t ys[K], ts[K];
      // low 32 bits of c at limb offset s, high 32 bits at s + 1
      shift_limbs(r1, s, ys);
      (void)submul(r0, ys, (uint32_t)c);
      shift_limbs(t1, s, ts);
      (void)submul(t0, ts, (uint32_t)c);
      if (c >> 32) {
        shift_limbs(r1, s + 1, ys);
        (void)submul(r0, ys, (uint32_t)(c >> 32));
        shift_limbs(t1, s + 1, ts);
        (void)submul(t0, ts, (uint32_t)(c >> 32));
      }
    }
  }
  // ---- checks and output: a = sign(t) r, b = |t|
  const bool neg = (t1[K - 1] >> 31) != 0;
  if (neg) negate(t1);
  bool ok = st == 0 && it < cap && !is_zero(t1) && cmp(t1, Bv) <= 0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    if (i < P) {
      const FpConst F = fpc(a.pc[i]);
      const int32_t c32m = fp_mul(a.pc[i].c32, a.pc[i].r2, F);  // 2^32 R mod p
      if (mod_prime(t1, F, c32m) == 0) ok = false;              // gcd(t, M) != 1
    }
  }
  if (ok && neg) negate(r1);
  const int L = a.L;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (k < L) {
      a.num[(int64_t)k * a.ld + q] = ok ? (int32_t)r1[k] : 0;
      a.den[(int64_t)k * a.ld + q] = ok ? t1[k] : 0u;
    }
  }
  if (a.status) a.status[q] = st ? st : (ok ? 0 : 1);
}

// ---------------------------------------------------------------------------
// host side: limb integers
// ---------------------------------------------------------------------------
using Big = std::vector<uint32_t>;  // little-endian limbs

void big_mul_small(Big& x, uint32_t m) {
  uint64_t carry = 0;
  for (auto& w : x) {
    const uint64_t s = (uint64_t)w * m + carry;
    w = (uint32_t)s;
    carry = s >> 32;
  }
  if (carry) x.push_back((uint32_t)carry);
}

int big_cmp(const Big& x, const Big& y) {
  const size_t n = x.size() > y.size() ? x.size() : y.size();
  for (size_t k = n; k-- > 0;) {
    const uint32_t a = k < x.size() ? x[k] : 0, b = k < y.size() ? y[k] : 0;
    if (a != b) return a > b ? 1 : -1;
  }
  return 0;
}

Big big_sq(const Big& x) {
  Big r(2 * x.size() + 1, 0);
  for (size_t i = 0; i < x.size(); ++i) {
    uint64_t carry = 0;
    for (size_t j = 0; j < x.size(); ++j) {
      const uint64_t s = (uint64_t)x[i] * x[j] + r[i + j] + carry;
      r[i + j] = (uint32_t)s;
      carry = s >> 32;
    }
    size_t k = i + x.size();
    while (carry) {
      const uint64_t s = (uint64_t)r[k] + carry;
      r[k++] = (uint32_t)s;
      carry = s >> 32;
    }
  }
  return r;
}

// floor(sqrt(N)), bit by bit from the top
Big big_isqrt(const Big& N) {
  size_t bits = N.size() * 32;
  Big root((N.size() + 1) / 2 + 1, 0);
  for (size_t b = bits / 2 + 1; b-- > 0;) {
    Big cand = root;
    cand[b / 32] |= 1u << (b % 32);
    if (big_cmp(big_sq(cand), N) <= 0) root = cand;
  }
  return root;
}

uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = (unsigned __int128)r * a % m;
    a = (unsigned __int128)a * a % m;
    e >>= 1;
  }
  return r;
}

int32_t bal(uint64_t x, uint64_t p) {
  x %= p;
  return x > (p - 1) / 2 ? (int32_t)((int64_t)x - (int64_t)p) : (int32_t)x;
}

}  // namespace
}  // namespace bg

extern "C" {

int bg_fp_from_rational(uint32_t p, int64_t count, const int64_t* num, const int64_t* den, uint32_t* out,
                        uint8_t* status, void* hip_stream) {
  if (p < 3 || p >= 0x80000000u || !bg::is_prime_u32(p)) return BG_ENOTPRIME;
  if (count < 0) return BG_EINVAL;
  if (count == 0) return BG_OK;
  if (!num || !den || !out) return BG_EINVAL;
  bg::ResidueArgs a{};
  a.num = num;
  a.den = den;
  a.out = out;
  a.status = status;
  a.count = count;
  a.fp = bg::make_fp_const(p);
  const uint64_t R = bg::powmod64(2, 64, p);
  a.r3 = bg::bal((unsigned __int128)R * R % p * R % p, p);
  const int64_t lanes = (count + bg::kResidueChunk - 1) / bg::kResidueChunk;
  const int64_t blocks = (lanes + 255) / 256;
  if (blocks > 0x7FFFFFFF) return BG_EINVAL;
  void* args[] = {&a};
  return hipLaunchKernel(reinterpret_cast<const void*>(&bg::residue_kernel), dim3((unsigned)blocks), dim3(256),
                         args, 0, static_cast<hipStream_t>(hip_stream)) == hipSuccess
             ? BG_OK
             : BG_EHIP;
}

int bg_rational_reconstruct(int nprimes, const uint32_t* primes, int64_t npts, int64_t ld,
                            const uint32_t* residues, int32_t* num, uint32_t* den, uint8_t* status,
                            void* hip_stream) {
  if (nprimes < 1 || nprimes > BG_RR_MAX_PRIMES || !primes) return BG_EINVAL;
  for (int i = 0; i < nprimes; ++i) {
    if (primes[i] < 3 || primes[i] >= 0x80000000u || !bg::is_prime_u32(primes[i])) return BG_ENOTPRIME;
    for (int j = 0; j < i; ++j)
      if (primes[j] == primes[i]) return BG_EINVAL;
  }
  if (npts < 0) return BG_EINVAL;
  if (npts == 0) return BG_OK;
  if (ld < npts || !residues || !num || !den) return BG_EINVAL;
  bg::RRArgs a{};
  memset(&a, 0, sizeof(a));
  a.residues = residues;
  a.num = num;
  a.den = den;
  a.status = status;
  a.npts = npts;
  a.ld = ld;
  a.nprimes = nprimes;
  a.L = BG_RR_LIMBS(nprimes);
  bg::Big M{1};
  for (int i = 0; i < nprimes; ++i) {
    const uint64_t p = primes[i];
    const bg::FpConst k = bg::make_fp_const((uint32_t)p);
    bg::PrimeConst& c = a.pc[i];
    c.p = k.p;
    c.h = k.h;
    c.c32 = k.c32;
    c.c64 = k.c64;
    c.pinv = k.pinv;
    const uint64_t R = bg::powmod64(2, 64, p);
    c.r2 = bg::bal((unsigned __int128)R * R % p, p);
    uint64_t prod = 1;  // p_0 ... p_{i-1} mod p_i
    for (int j = 0; j < i; ++j) prod = (unsigned __int128)prod * (primes[j] % p) % p;
    const uint64_t inv = bg::powmod64(prod, p - 2, p);
    c.minv = bg::bal((unsigned __int128)inv * R % p, p);
    bg::big_mul_small(M, (uint32_t)p);
  }
  bg::Big Mm1 = M;  // (M - 1) / 2; M is odd, so M - 1 only clears bit 0
  Mm1[0] -= 1;
  for (size_t k = 0; k < Mm1.size(); ++k) Mm1[k] = (Mm1[k] >> 1) | (k + 1 < Mm1.size() ? (Mm1[k + 1] << 31) : 0u);
  const bg::Big Bv = bg::big_isqrt(Mm1);
  for (size_t k = 0; k < M.size() && k < (size_t)BG_RR_MAX_PRIMES; ++k) a.M[k] = M[k];
  for (size_t k = 0; k < Bv.size() && k < (size_t)BG_RR_MAX_PRIMES; ++k) a.B[k] = Bv[k];
  const int64_t blocks = (npts + 255) / 256;
  if (blocks > 0x7FFFFFFF) return BG_EINVAL;
  const void* fn = nprimes <= 8    ? reinterpret_cast<const void*>(&bg::rr_kernel<8>)
                   : nprimes <= 16 ? reinterpret_cast<const void*>(&bg::rr_kernel<16>)
                                   : reinterpret_cast<const void*>(&bg::rr_kernel<32>);
  void* args[] = {&a};
  return hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(256), args, 0, static_cast<hipStream_t>(hip_stream)) ==
                 hipSuccess
             ? BG_OK
             : BG_EHIP;
}

}  // extern "C"
