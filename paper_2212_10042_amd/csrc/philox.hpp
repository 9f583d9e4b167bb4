// philox.hpp -- Philox4x32-10 counter-based generator for gfx950 device code.
//
// Salmon, Moraes, Dror & Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3"
// (SC'11), Section 3.3: ten rounds of the Philox S-box on four 32-bit words,
// multipliers 0xD2511F53 / 0xCD9E8D57, key schedule bumped by 0x9E3779B9 /
// 0xBB67AE85 between rounds.  The stream used by this library is
//   word(seed, k, w) = Philox4x32-10(key = (seed lo, seed hi), ctr = (w/4, k, 0, 0))[w mod 4]
// so a simulation's words do not depend on the tile (common random numbers).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cse {

struct u32x4 {
    uint32_t x, y, z, w;
};

// One round: two 32x32->64 products (v_mad_u64_u32 on CDNA), two 3-way xors.
__device__ __forceinline__ void philox_round(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                             uint32_t k0, uint32_t k1) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
}

// Block `blk` of simulation `sim`: counter (blk, sim, 0, 0).
__device__ __forceinline__ u32x4 philox_block(uint32_t blk, uint32_t sim, uint32_t k0, uint32_t k1) {
    uint32_t c0 = blk, c1 = sim, c2 = 0u, c3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        philox_round(c0, c1, c2, c3, k0, k1);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return u32x4{c0, c1, c2, c3};
}

// The uniform adjoined to simulation `sim` by the randomised test: first word of the block at
// counter (0, sim, 1, 0).  Data blocks have counter word 2 = 0, so the two streams never meet.
__device__ __forceinline__ uint32_t philox_tiebreak(uint32_t sim, uint32_t k0, uint32_t k1) {
    uint32_t c0 = 0u, c1 = sim, c2 = 1u, c3 = 0u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        philox_round(c0, c1, c2, c3, k0, k1);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

__device__ __forceinline__ uint32_t u32x4_get(const u32x4 &v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

}  // namespace cse
