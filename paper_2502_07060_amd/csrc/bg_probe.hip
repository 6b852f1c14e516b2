// Issue-rate probe: lane-operations per second of the VALU instructions the
// recursion kernels are built from, measured on the device at hand.  The Z_p
// path's arithmetic is 64-bit integer multiply-add modulo p < 2^31 (paper
// Sec. 3); its roofline is the issue rate of the 32x32 -> 64-bit integer
// multiply-add, which has no published peak, so this measures it next to the
// FP64 FMA whose peak is published.
//
// Each lane runs CHAINS independent dependency chains of one instruction for
// `iters` rounds; many waves per SIMD hide the latency of each chain, so the
// launch is bound by issue.  The loop-carried operand (the low word of the
// accumulator, or the accumulator itself) keeps the compiler from hoisting or
// folding the arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bg.h"

namespace {

constexpr int kChains = 8;
constexpr int kBlock = 256;

template <int KIND>
__global__ __launch_bounds__(kBlock) void issue_kernel(uint64_t* sink, int iters, uint32_t seed) {
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t b = seed | 1u;
  uint64_t acc[kChains];
  double facc[kChains];
  uint32_t x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    acc[c] = (uint64_t)(t * 2654435761u + c);
    facc[c] = (double)(t + c) * 0x1.0p-20;
    x[c] = t ^ (0x9E3779B9u * (c + 1));
  }
#pragma unroll 4
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (KIND == BG_PROBE_MAD_I64_I32) {
        // v_mad_i64_i32: (int64)(int32)acc * (int32)b + acc
        acc[c] = (uint64_t)((int64_t)(int32_t)(uint32_t)acc[c] * (int64_t)(int32_t)b) + acc[c];
      } else if constexpr (KIND == BG_PROBE_MAD_U64_U32) {
        acc[c] = (uint64_t)(uint32_t)acc[c] * (uint64_t)b + acc[c];
      } else if constexpr (KIND == BG_PROBE_FMA_F64) {
        facc[c] = __builtin_fma(facc[c], 0.9999999, 0x1.0p-30);
      } else if constexpr (KIND == BG_PROBE_MUL_LO_U32) {
        // a squaring chain: a constant factor would let the compiler merge
        // the unrolled rounds (x b b b b = x b^4) and count one multiply as four
        x[c] = x[c] * x[c];
      } else {  // BG_PROBE_DPP_MOV_B32
        // row_ror:1 (a pair swap applied twice is the identity, which the
        // compiler removes)
        x[c] = (uint32_t)__builtin_amdgcn_mov_dpp((int)x[c], 0x121, 0xF, 0xF, false);
      }
    }
  }
  uint64_t r = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) r += acc[c] + (uint64_t)__builtin_bit_cast(uint64_t, facc[c]) + x[c];
  sink[t] = r;
}

template <int KIND>
hipError_t launch(uint64_t* sink, int blocks, int iters, uint32_t seed, hipStream_t st) {
  hipLaunchKernelGGL(issue_kernel<KIND>, dim3(blocks), dim3(kBlock), 0, st, sink, iters, seed);
  return hipGetLastError();
}

hipError_t launch_kind(int kind, uint64_t* sink, int blocks, int iters, uint32_t seed, hipStream_t st) {
  switch (kind) {
    case BG_PROBE_MAD_I64_I32: return launch<BG_PROBE_MAD_I64_I32>(sink, blocks, iters, seed, st);
    case BG_PROBE_MAD_U64_U32: return launch<BG_PROBE_MAD_U64_U32>(sink, blocks, iters, seed, st);
    case BG_PROBE_FMA_F64: return launch<BG_PROBE_FMA_F64>(sink, blocks, iters, seed, st);
    case BG_PROBE_MUL_LO_U32: return launch<BG_PROBE_MUL_LO_U32>(sink, blocks, iters, seed, st);
    default: return launch<BG_PROBE_DPP_MOV_B32>(sink, blocks, iters, seed, st);
  }
}

}  // namespace

extern "C" int bg_issue_rate(int kind, int blocks, int iters, int reps, double* lane_ops_per_s, double* ms_per_launch,
                             void* hip_stream) {
  if (kind < BG_PROBE_MAD_I64_I32 || kind > BG_PROBE_DPP_MOV_B32) return BG_EINVAL;
  if (blocks <= 0 || blocks > (1 << 20) || iters <= 0 || reps <= 0 || !lane_ops_per_s) return BG_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  uint64_t* sink = nullptr;
  if (hipMalloc(&sink, (size_t)blocks * kBlock * sizeof(uint64_t)) != hipSuccess) return BG_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = BG_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = BG_EHIP;
  if (rc == BG_OK && launch_kind(kind, sink, blocks, iters, 12345u, st) != hipSuccess) rc = BG_EHIP;  // warm-up
  float ms = 0.f;
  if (rc == BG_OK && hipEventRecord(e0, st) != hipSuccess) rc = BG_EHIP;
  for (int r = 0; r < reps && rc == BG_OK; ++r)
    if (launch_kind(kind, sink, blocks, iters, 12345u + r, st) != hipSuccess) rc = BG_EHIP;
  if (rc == BG_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                      hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = BG_EHIP;
  if (rc == BG_OK) {
    const double per = (double)ms / reps;
    const double ops = (double)blocks * kBlock * (double)iters * kChains;
    *lane_ops_per_s = ops / (per * 1e-3);
    if (ms_per_launch) *ms_per_launch = per;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  return rc;
}
