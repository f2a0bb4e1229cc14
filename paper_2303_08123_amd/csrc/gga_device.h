// Device helpers shared by the library's kernels: Philox4x32-10 and wave-wide
// lane shifts.  gfx950 (CDNA4) only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gga {

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11, Section 4):
// per round two 32x32->64 products of counter words 0 and 2 with fixed odd
// multipliers; the new counter is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0) and
// the key advances by a Weyl increment between rounds.  The key is uniform
// across a wave in every use here, so its schedule stays in scalar registers.
struct Block4 { uint32_t w0, w1, w2, w3; };

__device__ __forceinline__ Block4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Whole-wave lane shifts through DPP (GFX9 wave_shr:1 / wave_shl:1).  Lanes
// whose source lies outside the wave read 0 (bound_ctrl), which the callers
// use as "no neighbour".  The move folds into the consuming VALU op.
__device__ __forceinline__ float lane_from_left(float v) {   // lane l <- lane l-1
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_from_right(float v) {  // lane l <- lane l+1
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        0, __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

__device__ __forceinline__ uint32_t lane_from_left_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t lane_from_right_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, true);
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace gga
