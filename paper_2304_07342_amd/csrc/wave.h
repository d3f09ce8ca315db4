// Wavefront-64 primitives for CDNA (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpulz {

template <int S> struct SymType;
template <> struct SymType<1> { using T = uint8_t; };
template <> struct SymType<2> { using T = uint16_t; };
template <> struct SymType<4> { using T = uint32_t; };
template <> struct SymType<8> { using T = uint64_t; };

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// 64-bit mask of the lanes whose predicate holds (a v_cmp result in SGPRs).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of set bits of `m` below this lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}

// Inclusive prefix sum across the wave, in registers (DPP): shifts by 1, 2,
// 4 and 8 lanes within each 16-lane row (lanes shifted in from outside the
// row read 0), then the GFX9 row broadcasts add row 0's total to row 1, row
// 2's to row 3, and lane 31's running total to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, true);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, true);  // row_bcast:31
  return x;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}

// Maximum of `v` over the wave, returned as a wave-uniform value. DPP steps:
// swap pairs, swap pairs of pairs, mirror within 8 and 16 lanes (every lane
// then holds its 16-lane row's maximum), then the GFX9 row broadcasts fold
// row 0 into row 1, row 2 into row 3, and lane 31 into rows 2 and 3, so lane
// 63 holds the maximum of all four rows. Lanes a step does not write read 0,
// the identity of an unsigned maximum, which lets each move fold into the
// v_max as a DPP operand.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, true));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, true));
  return readlane(v, 63);
}

// Orders this wave's LDS and global accesses before the ones that follow
// (LDS is accessed in order within a wave; this keeps the compiler from
// moving accesses across the point and waits for outstanding ones).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

}  // namespace gpulz
