// Standalone batched Z_p operations (paper Sec. 3: the finite-field library
// that the recursion is built on, usable on its own): tensor contraction over
// any group of indices, with the second operand per event or shared, and
// division.  Residues are canonical uint32 in [0, p); the event index is the
// fastest one in every array (element e of event q at e * ld + q), as in the
// amplitude entry points, so the lanes of a wave read consecutive words.
//
// Contraction, one event per lane: z[i][k] = sum_j x[i][j] y[j][k].  Values
// are taken as balanced representatives (|v| <= (p-1)/2), so a product is
// below 2^60 and four of them fit beside a folded accumulator (field_fp.h);
// each output is reduced once at the end (REDC2 and one product with R^2).
// Outputs are computed eight columns k at a time, so every x[i][j] is read
// once per eight outputs; repeated reads of an event's operands hit the
// caches (the algorithmic traffic is read once).
//
// Division: Montgomery batch inversion over 16 values per lane (one Fermat
// power per 16 quotients).
//
// Small contractions (J, K <= 8) have a kernel of their own that reads y once
// per event into registers (static 8 x 8 slots, guarded by the run-time
// sizes) and each x[i][j] once.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "bg.h"
#include "bg_registry.h"
#include "field_fp.h"

namespace bg {
namespace {

constexpr int kKBlock = 8;
constexpr int kDivChunk = 16;

struct ContractArgs {
  const uint32_t* x;
  const uint32_t* y;
  uint32_t* z;
  uint8_t* status;
  int64_t npts, ld;
  int I, J, K;
  int y_batched;
  FpConst fp;
  int32_t r2;  // R^2 mod p, balanced
};

__device__ __forceinline__ int32_t bal_of(uint32_t v, const FpConst& F, uint32_t& maxraw) {
  maxraw = maxraw > v ? maxraw : v;
  return fp_from_canonical(v < (uint32_t)F.p ? v : 0u, F);
}

__global__ __launch_bounds__(256) void contract_kernel(ContractArgs a) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= a.npts) return;
  const FpConst& F = a.fp;
  const int64_t ys = a.y_batched ? a.ld : 1;   // element stride of y ([J][K][ld] or [J][K])
  const int64_t yq = a.y_batched ? q : 0;
  uint32_t maxraw = 0;
  // a pass over the inputs finds non-canonical residues first, so that the
  // outputs of such an event are all sentinels
  for (int e = 0; e < a.I * a.J; ++e) maxraw = max(maxraw, a.x[(int64_t)e * a.ld + q]);
  for (int e = 0; e < a.J * a.K; ++e) maxraw = max(maxraw, a.y[(int64_t)e * ys + yq]);
  const bool bad = maxraw >= (uint32_t)F.p;
  for (int i = 0; i < a.I; ++i) {
    for (int k0 = 0; k0 < a.K; k0 += kKBlock) {
      int64_t acc[kKBlock];
#pragma unroll
      for (int u = 0; u < kKBlock; ++u) acc[u] = 0;
      uint32_t dummy = 0;
      int j = 0;
      for (; j < a.J; ++j) {
        const int32_t xv = bal_of(a.x[((int64_t)i * a.J + j) * a.ld + q], F, dummy);
#pragma unroll
        for (int u = 0; u < kKBlock; ++u) {
          if (k0 + u < a.K) {
            const int32_t yv = bal_of(a.y[((int64_t)j * a.K + k0 + u) * ys + yq], F, dummy);
            acc[u] = mad64(xv, yv, acc[u]);
          }
        }
        if ((j & 3) == 3) {  // four products of < 2^60 beside a folded accumulator
#pragma unroll
          for (int u = 0; u < kKBlock; ++u) acc[u] = fp_fold(acc[u], F);
        }
      }
#pragma unroll
      for (int u = 0; u < kKBlock; ++u) {
        if (k0 + u < a.K) {
          const int32_t s = fp_mul(fp_redc2(fp_fold(acc[u], F), F), a.r2, F);  // sum R^-1 R^2 R^-1
          a.z[((int64_t)i * a.K + k0 + u) * a.ld + q] = bad ? 0xFFFFFFFFu : fp_to_canonical(s, F);
        }
      }
    }
  }
  if (a.status) a.status[q] = bad ? PT_BADRESIDUE : PT_OK;
}

// J, K <= kSmall: y in registers, every input read once
constexpr int kSmall = 8;

__global__ __launch_bounds__(256) void contract_small_kernel(ContractArgs a) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= a.npts) return;
  const FpConst& F = a.fp;
  const int64_t ys = a.y_batched ? a.ld : 1;
  const int64_t yq = a.y_batched ? q : 0;
  uint32_t maxraw = 0;
  int32_t yv[kSmall][kSmall];
#pragma unroll
  for (int j = 0; j < kSmall; ++j)
#pragma unroll
    for (int k = 0; k < kSmall; ++k)
      yv[j][k] = (j < a.J && k < a.K) ? bal_of(a.y[((int64_t)j * a.K + k) * ys + yq], F, maxraw) : 0;
  // outputs go out as they are made; an event with a non-canonical input is
  // overwritten with sentinels afterwards
  for (int i = 0; i < a.I; ++i) {
    int32_t xv[kSmall];
#pragma unroll
    for (int j = 0; j < kSmall; ++j) xv[j] = j < a.J ? bal_of(a.x[((int64_t)i * a.J + j) * a.ld + q], F, maxraw) : 0;
#pragma unroll
    for (int k = 0; k < kSmall; ++k) {
      if (k < a.K) {
        int64_t acc = 0;
#pragma unroll
        for (int j = 0; j < kSmall; ++j) {
          acc = mad64(xv[j], yv[j][k], acc);  // zero slots add nothing
          if (j == 3) acc = fp_fold(acc, F);
        }
        const int32_t s = fp_mul(fp_redc2(fp_fold(acc, F), F), a.r2, F);
        a.z[((int64_t)i * a.K + k) * a.ld + q] = fp_to_canonical(s, F);
      }
    }
  }
  const bool bad = maxraw >= (uint32_t)F.p;
  if (bad)
    for (int e = 0; e < a.I * a.K; ++e) a.z[(int64_t)e * a.ld + q] = 0xFFFFFFFFu;
  if (a.status) a.status[q] = bad ? PT_BADRESIDUE : PT_OK;
}

struct DivideArgs {
  const uint32_t* x;
  const uint32_t* y;
  uint32_t* z;
  uint8_t* status;
  int64_t count;
  uint32_t yscalar;  // used when y == nullptr: its inverse times R (Montgomery form)
  FpConst fp;
  int32_t r2;
};

// Lane t of block b takes the values b 4096 + u 256 + t, u < 16: each of the
// 16 loads of a wave reads 256 consecutive bytes.
__global__ __launch_bounds__(256) void divide_kernel(DivideArgs a) {
  const int64_t base = (int64_t)blockIdx.x * 256 * kDivChunk + threadIdx.x;
  const FpConst& F = a.fp;
  int32_t xm[kDivChunk], ym[kDivChunk];
  uint8_t st[kDivChunk];
  int32_t acc = F.one;
#pragma unroll
  for (int u = 0; u < kDivChunk; ++u) {
    const int64_t e = base + (int64_t)u * 256;
    if (e < a.count) {
      const uint32_t xr = a.x[e];
      const uint32_t yr = a.y ? a.y[e] : 1u;
      st[u] = (xr >= (uint32_t)F.p || yr >= (uint32_t)F.p) ? PT_BADRESIDUE : PT_OK;
      xm[u] = fp_mul(fp_from_canonical(xr < (uint32_t)F.p ? xr : 0u, F), a.r2, F);  // x R
      ym[u] = a.y ? fp_mul(fp_from_canonical(yr < (uint32_t)F.p ? yr : 0u, F), a.r2, F) : F.one;
      if (st[u] == PT_OK && ym[u] == 0) st[u] = PT_SINGULAR;
      if (ym[u] == 0) ym[u] = F.one;
      xm[u] = fp_mul(xm[u], acc, F);  // x_u (y_0 ... y_{u-1})
      acc = fp_mul(acc, ym[u], F);
    }
  }
  int32_t inv = a.y ? fp_pow(acc, (uint32_t)(F.p - 2), F) : (int32_t)a.yscalar;
#pragma unroll
  for (int u = kDivChunk - 1; u >= 0; --u) {
    const int64_t e = base + (int64_t)u * 256;
    if (e < a.count) {
      const int32_t qv = fp_mul(xm[u], inv, F);
      inv = fp_mul(inv, ym[u], F);
      const int32_t v = fp_redc2((int64_t)qv, F);
      a.z[e] = st[u] == PT_OK ? fp_to_canonical(v, F) : 0xFFFFFFFFu;
      if (a.status) a.status[e] = st[u];
    }
  }
}

uint64_t powmod_u64(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = (unsigned __int128)r * a % m;
    a = (unsigned __int128)a * a % m;
    e >>= 1;
  }
  return r;
}

int32_t balanced_of(uint64_t x, uint64_t p) {
  x %= p;
  return x > (p - 1) / 2 ? (int32_t)((int64_t)x - (int64_t)p) : (int32_t)x;
}

int32_t r2_of(uint32_t p) {
  const uint64_t R = powmod_u64(2, 64, p);
  return balanced_of((unsigned __int128)R * R % p, p);
}

}  // namespace
}  // namespace bg

extern "C" {

int bg_fp_contract(uint32_t p, int I, int J, int K, int64_t npts, int64_t ld, const uint32_t* x,
                   const uint32_t* y, int y_batched, uint32_t* z, uint8_t* status, void* hip_stream) {
  if (p < 3 || p >= 0x80000000u || !bg::is_prime_u32(p)) return BG_ENOTPRIME;
  if (I < 1 || J < 1 || K < 1 || I > BG_FP_MAX_DIM || J > BG_FP_MAX_DIM || K > BG_FP_MAX_DIM) return BG_EDOMAIN;
  if (npts < 0) return BG_EINVAL;
  if (npts == 0) return BG_OK;
  if (ld < npts || !x || !y || !z) return BG_EINVAL;
  bg::ContractArgs a{};
  a.x = x;
  a.y = y;
  a.z = z;
  a.status = status;
  a.npts = npts;
  a.ld = ld;
  a.I = I;
  a.J = J;
  a.K = K;
  a.y_batched = y_batched ? 1 : 0;
  a.fp = bg::make_fp_const(p);
  a.r2 = bg::r2_of(p);
  const int64_t blocks = (npts + 255) / 256;
  if (blocks > 0x7FFFFFFF) return BG_EINVAL;
  void* args[] = {&a};
  const void* fn = (J <= bg::kSmall && K <= bg::kSmall) ? reinterpret_cast<const void*>(&bg::contract_small_kernel)
                                                        : reinterpret_cast<const void*>(&bg::contract_kernel);
  return hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(256),
                         args, 0, static_cast<hipStream_t>(hip_stream)) == hipSuccess
             ? BG_OK
             : BG_EHIP;
}

static int launch_divide(uint32_t p, int64_t count, const uint32_t* x, const uint32_t* y, uint32_t yscalar,
                         uint32_t* z, uint8_t* status, void* hip_stream) {
  bg::DivideArgs a{};
  a.x = x;
  a.y = y;
  a.z = z;
  a.status = status;
  a.count = count;
  a.fp = bg::make_fp_const(p);
  a.r2 = bg::r2_of(p);
  if (!y) {  // (1 / y) R mod p, balanced
    const uint64_t inv = bg::powmod_u64(yscalar, p - 2, p);
    const uint64_t R = bg::powmod_u64(2, 64, p);
    a.yscalar = (uint32_t)bg::balanced_of((unsigned __int128)inv * R % p, p);
  }
  const int64_t blocks = (count + 256 * bg::kDivChunk - 1) / (256 * bg::kDivChunk);
  if (blocks > 0x7FFFFFFF) return BG_EINVAL;
  void* args[] = {&a};
  return hipLaunchKernel(reinterpret_cast<const void*>(&bg::divide_kernel), dim3((unsigned)blocks), dim3(256),
                         args, 0, static_cast<hipStream_t>(hip_stream)) == hipSuccess
             ? BG_OK
             : BG_EHIP;
}

int bg_fp_divide(uint32_t p, int64_t count, const uint32_t* x, const uint32_t* y, uint32_t* z, uint8_t* status,
                 void* hip_stream) {
  if (p < 3 || p >= 0x80000000u || !bg::is_prime_u32(p)) return BG_ENOTPRIME;
  if (count < 0) return BG_EINVAL;
  if (count == 0) return BG_OK;
  if (!x || !y || !z) return BG_EINVAL;
  return launch_divide(p, count, x, y, 0, z, status, hip_stream);
}

int bg_fp_divide_scalar(uint32_t p, int64_t count, const uint32_t* x, uint32_t y, uint32_t* z, uint8_t* status,
                        void* hip_stream) {
  if (p < 3 || p >= 0x80000000u || !bg::is_prime_u32(p)) return BG_ENOTPRIME;
  if (y >= p) return BG_EINVAL;
  if (y == 0) return BG_EDOMAIN;  // no inverse
  if (count < 0) return BG_EINVAL;
  if (count == 0) return BG_OK;
  if (!x || !z) return BG_EINVAL;
  return launch_divide(p, count, x, nullptr, y, z, status, hip_stream);
}

}  // extern "C"
