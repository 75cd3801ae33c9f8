// Cross-lane sums for gfx950 wavefronts (wave64): DPP row moves, no LDS
// round trip. Used by every kernel that reduces over a lane group.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgm {
namespace {

// Lane exchange inside one DPP row of 16 lanes (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), CTRL, 0xF, 0xF, false));
  const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), CTRL, 0xF, 0xF, false));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within each 8
constexpr int kDppMirror = 0x140;      // lane i <- 15 - i within each 16

// Sum over each aligned group of G consecutive lanes (G = 1, 2, 4, 8, 16);
// every lane of the group gets the same bits. All lanes of a group must be
// active. Each stage adds two partial sums over disjoint lane sets.
template <int G, typename S>
__device__ __forceinline__ S group_sum(S v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
  if constexpr (G >= 16) v += dpp_mov<kDppMirror>(v);
  if constexpr (G >= 8) v += dpp_mov<kDppHalfMirror>(v);
  if constexpr (G >= 4) v += dpp_mov<kDppXor2>(v);
  if constexpr (G >= 2) v += dpp_mov<kDppXor1>(v);
  return v;
}

}  // namespace
}  // namespace mgm
