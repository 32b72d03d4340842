// wave.hpp -- wavefront-wide reductions of 32-bit values over the 64 lanes
// of a gfx950 wavefront, with DPP row operations: quad permutations, the
// half-row and row mirrors, then the row broadcasts of lanes 15 and 31
// (gfx9 DPP), after which lane 63 holds the result of every lane.  Every
// lane must be active (the row broadcasts read lanes of other rows).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace qd {

// DPP controls (gfx9): quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror,
// row_mirror, row_bcast:15, row_bcast:31.
constexpr int kDppQuadSwap1 = 0xB1, kDppQuadSwap2 = 0x4E;
constexpr int kDppRowHalfMirror = 0x141, kDppRowMirror = 0x140;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_move(uint32_t identity, uint32_t v) {
  // Lanes whose row is masked out or whose source is invalid keep `identity`.
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(static_cast<int>(identity), static_cast<int>(v), CTRL,
                                                           ROW_MASK, 0xF, false));
}

// op(a, b) is associative and commutative; identity is its neutral value.
template <typename Op>
__device__ __forceinline__ uint32_t wave_reduce_dpp(uint32_t v, uint32_t identity, Op op) {
  v = op(v, dpp_move<kDppQuadSwap1, 0xF>(identity, v));
  v = op(v, dpp_move<kDppQuadSwap2, 0xF>(identity, v));      // every lane: its quad
  v = op(v, dpp_move<kDppRowHalfMirror, 0xF>(identity, v));  // its half row (8 lanes)
  v = op(v, dpp_move<kDppRowMirror, 0xF>(identity, v));      // its row (16 lanes)
  v = op(v, dpp_move<kDppRowBcast15, 0xA>(identity, v));     // rows 1, 3: with rows 0, 2
  v = op(v, dpp_move<kDppRowBcast31, 0xC>(identity, v));     // rows 2, 3: with lane 31
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  return wave_reduce_dpp(v, 0xFFFFFFFFu, [](uint32_t a, uint32_t b) { return a < b ? a : b; });
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  return wave_reduce_dpp(v, 0u, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  return wave_reduce_dpp(v, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}

// Index of the last of n ascending keys (key(0) <= x) that is <= x, found
// with one or two rounds of loads spread over the wavefront's lanes (the
// keys of a chunk of 64, after those of every 64th key when n > 64)
// instead of a chain of log2(n) dependent loads.  n <= 4096 (larger: a
// binary search).  Every lane must be active; the result is uniform.
template <typename Key>
__device__ __forceinline__ int wave_last_le(int n, unsigned long long x, Key key) {
  if (n > 64 * 64) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (key(mid) <= x) lo = mid;
      else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
  }
  const int lane = static_cast<int>(threadIdx.x & 63);
  int chunk = 0;
  if (n > 64) {
    const int i = lane * 64;
    chunk = __builtin_amdgcn_readfirstlane(__popcll(__ballot(i < n && key(i) <= x)) - 1);
  }
  const int i = chunk * 64 + lane;
  return __builtin_amdgcn_readfirstlane(chunk * 64 + __popcll(__ballot(i < n && key(i) <= x)) - 1);
}

}  // namespace qd
