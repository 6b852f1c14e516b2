// Shared compile-time helpers for the Berends-Giele kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

namespace bg {

// ---------------------------------------------------------------------------
// compile-time loops: body(std::integral_constant<int, I>) for I in [B, E)
// ---------------------------------------------------------------------------
template <int B, int... Is, class F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, B + Is>{}), ...);
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (E > B) static_for_impl<B>(std::make_integer_sequence<int, E - B>{}, f);
}

// ---------------------------------------------------------------------------
// XCD-aware block order.  The workgroups of a launch go to the device's 8
// XCDs in turn (workgroup b to XCD b mod 8), and each XCD has its own L2.  A
// kernel whose block reads less than a cache line of every input row (a few
// points per block, the point index fastest in memory) renumbers its blocks
// so that consecutive point ranges run on one XCD: the blocks that share a
// line then share one L2, and the line comes from HBM once instead of once
// per XCD.  The renumbering is a bijection of [0, gridDim.x) whatever the
// hardware's actual placement, so it affects only where data is cached.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xcd_block_index() {
  constexpr uint32_t X = 8;
  const uint32_t b = blockIdx.x, nb = gridDim.x;
  const uint32_t per = nb / X, rem = nb % X;
  const uint32_t x = b % X, k = b / X;
  return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// ---------------------------------------------------------------------------
// sub-range bookkeeping for N = n - 1 legs (0-based i <= j < N)
// ---------------------------------------------------------------------------
template <int N>
struct Ranges {
  // ranges ordered by length, then left end: [0..0],[1..1],...,[0..1],[1..2],...
  static constexpr int count = N * (N + 1) / 2;
  static constexpr int idx(int i, int j) {
    // number of ranges of length < L is sum_{l<L} (N - l + 1) = (L-1)(2N - L + 2)/2
    return ((j - i) * (2 * N - (j - i) + 1)) / 2 + i;
  }
  // ranges of length >= 2 that need a propagator (all but the root)
  static constexpr int nprop = N * (N - 1) / 2 - 1 > 0 ? N * (N - 1) / 2 - 1 : 0;
  static constexpr int pidx(int i, int j) { return idx(i, j) - N; }  // length >= 2 only
  // number of non-root currents
  static constexpr int ncur = count - 1;
};

// ---------------------------------------------------------------------------
// cross-lane sums inside groups of L consecutive lanes (L = 1, 2, 4, 8, 16)
// via DPP row permutations; every lane of a group ends with the group sum.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// the two halves move separately and are reassembled as a register pair (an
// OR of shifted halves would be turned into two 64-bit additions downstream)
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const u32x2 x = __builtin_bit_cast(u32x2, v);
  u32x2 r;
  r.x = dpp_u32<CTRL>(x.x);
  r.y = dpp_u32<CTRL>(x.y);
  return __builtin_bit_cast(uint64_t, r);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  return __builtin_bit_cast(double, dpp_u64<CTRL>(__builtin_bit_cast(uint64_t, v)));
}

// DPP controls (GFX9 encoding): quad_perm [1,0,3,2], [2,3,0,1],
// row_half_mirror, row_mirror.
constexpr int DPP_QP_1032 = 0xB1;
constexpr int DPP_QP_2301 = 0x4E;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;

template <int L, class T, class Add, class Xchg>
__device__ __forceinline__ T group_sum(T v, Add add, Xchg xchg) {
  if constexpr (L >= 2) v = add(v, xchg(std::integral_constant<int, DPP_QP_1032>{}, v));
  if constexpr (L >= 4) v = add(v, xchg(std::integral_constant<int, DPP_QP_2301>{}, v));
  if constexpr (L >= 8) v = add(v, xchg(std::integral_constant<int, DPP_ROW_HALF_MIRROR>{}, v));
  if constexpr (L >= 16) v = add(v, xchg(std::integral_constant<int, DPP_ROW_MIRROR>{}, v));
  return v;
}

}  // namespace bg
