// k_sim.hip -- fused Monte Carlo kernels for gfx950.
//
// One wave owns one tile batch for a range of simulations.  Per simulation (one per lane)
// the Philox words are generated in registers, turned into draws, shared by every tile
// of the batch (common random numbers, Section 7.3), and reduced into per-tile rejection
// counts R and score sums (sufficient statistic over rejections, Example 1).  In
// calibration mode the 2-arm kernel also stores, per (simulation, batch), the 16 success
// counts from which every tile's outcome follows (one 16-byte record for 64 tiles), and the
// z-test each (simulation, tile)'s statistic S in float32.  Nothing else reaches memory.
#include "cse_internal.h"
#include "kernels.h"
#include "philox.hpp"

namespace cse {

// Lanes of one wave exchange values through LDS between these two points.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------------------------
// 2-arm binomial, n = 35 per arm, pooled z.  Words 0..34 are arm 0, 35..69 arm 1
// (18 Philox blocks).  Each wave's batch is an 8 x 8 product of thresholds: the success
// counts y0[u], y1[v] at 16 thresholds give the outcomes of all 64 tiles.  The 16 waves of a
// workgroup run the 16 batches of a 4 x 4 square of the threshold grid over the same
// simulations (wave 4 r + c: row group r, column group c): the Philox blocks of two chunks at a
// time (36) are generated once into LDS (two or three per wave), and the square's eight sets
// of 8 thresholds (four arm-0 row groups, four arm-1 column groups) are each counted once per
// simulation, by a pair of waves over the two halves of the arm's 35 words; the partial counts
// (8 bytes per simulation, a byte per threshold) go through LDS, and a batch adds the two
// halves of its row set and of its column set (bytes stay below 36: no carries).  Rejection at
// the design's cut is y1 >= c(y0) (z is increasing in y1 for fixed y0; checked on the host).
//
// In calibration mode each lane also writes its simulation's record (Rec2: y0[0..7], y1[0..7] as
// bytes, 16 bytes; a wave stores 1 KB contiguous per chunk).
//
// Per-lane accumulators are packed per tile: bits 0-5 rejections, 6-17 sum of y0 over
// rejections, 18-29 sum of y1 over rejections; exact for up to 63 simulations per lane
// between flushes (63 * 35 < 4096).  A flush transposes the 64 x 64 (lane, tile) matrix through
// LDS in two halves of 32 tiles, lanes l and l + 32 each summing half of tile l's column into
// 32-bit totals (joined by one shuffle at the end); the final totals are added to global
// memory with integer atomics (order-independent, hence deterministic).  The word buffer and
// the transpose buffers share 130 KB of LDS (workgroup barriers separate their uses): one
// workgroup of 16 waves per CU, four waves per SIMD.
// ------------------------------------------------------------------------------------
constexpr int WG2 = SQ2W * WAVE;   // 1024 threads
template <bool KEYS>
__global__ __launch_bounds__(WG2) void k_binom2(const Blk2 *__restrict__ blocks,
                                                const SquareItem *__restrict__ items,
                                                int64_t n_items, uint32_t key0, uint32_t key1,
                                                const int32_t *__restrict__ cut_tbl,
                                                uint32_t *__restrict__ R,
                                                unsigned long long *__restrict__ sumT,
                                                uint4 *__restrict__ recs) {
    constexpr int NT = B2U * B2V;
    constexpr int NW = 2 * NP35;
    constexpr int NB = (NW + 3) / 4;
    constexpr int NWAVES = SQ2W;
    constexpr int HALF = NT / 2;   // slots per flush half
    constexpr int JH = (NP35 + 1) / 2;   // words of the first counting half (18; the second 17)
    // flush transposes (per wave HALF x (64 + 1) words, padded against bank conflicts); between
    // flushes the same memory holds the chunk's Philox words
    // Two chunks per barrier phase: their 36 Philox blocks spread over the 16 waves (at most three
    // per wave, against two of one chunk's 18 on waves 0 and 1 while the other 14 wait), and half
    // the barriers.
    constexpr int CPB = 2;
    __shared__ uint32_t lds[NWAVES][HALF][WAVE + 1];
    __shared__ int32_t s_cut[64];
    __shared__ uint2 cnt[CPB][NWAVES][WAVE];   // per chunk, counting wave and lane: its 8 partial counts as bytes
    uint32_t(*words)[WAVE] = reinterpret_cast<uint32_t(*)[WAVE]>(&lds[0][0][0]);   // [CPB][4*NB][64]
    static_assert(CPB * 4 * NB * WAVE <= NWAVES * HALF * (WAVE + 1), "word buffer must fit");
    static_assert(CPB * NB <= 3 * NWAVES, "at most three Philox blocks per wave");

    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (threadIdx.x < 64) s_cut[threadIdx.x] = threadIdx.x <= NP35 ? cut_tbl[threadIdx.x] : 64;
    const int64_t it = blockIdx.x;
    if (it >= n_items) return;   // uniform over the workgroup
    const SquareItem *__restrict__ G = items + it;
    const int32_t blk = G->blk[wv];   // read in place: a register copy indexed by wv would go to scratch
    const bool live = blk >= 0;       // this wave's batch (row group wv >> 2, column group wv & 3)
    const Blk2 *__restrict__ B = blocks + (live ? blk : 0);   // dereferenced only when live
    const uint32_t kb = G->k_begin, ke = G->k_end;
    // counting set of this wave: set cs = wv >> 1 (0..3: arm 0, row group cs; 4..7: arm 1, column
    // group cs - 4) over word half wv & 1; thresholds from a block of the square that has them
    const int cs = wv >> 1, carm = cs >> 2, cgrp = cs & 3, chalf = wv & 1;
    int32_t csrc = -1;
    for (int i = 0; i < SQ2; ++i) {   // uniform
        const int32_t b = carm == 0 ? G->blk[cgrp * SQ2 + i] : G->blk[i * SQ2 + cgrp];
        if (csrc < 0 && b >= 0) csrc = b;
    }
    const bool counting = csrc >= 0;   // false: no batch of the square uses this set
    uint32_t Tc[B2U];
#pragma unroll
    for (int u = 0; u < B2U; ++u) Tc[u] = counting ? (carm == 0 ? blocks[csrc].T0[u] : blocks[csrc].T1[u]) : 0u;
    const int jw0 = carm * NP35 + (chalf ? JH : 0);   // first word of this wave's half
    const int jn = chalf ? NP35 - JH : JH;            // its word count
    uint4 *__restrict__ rbase = recs + ((KEYS && live) ? B->key_base : 0);
    const int rsrc = (wv >> 2) * 2, csrc2 = 2 * (SQ2 + (wv & 3));   // counting waves of this batch's sets

    uint32_t acc[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) acc[s] = 0u;
    // lane l: partial totals (over the lanes of half l >> 5) of slots l & 31 ([0]) and 32 + (l & 31) ([1])
    uint32_t totR[2] = {0u, 0u}, tot0[2] = {0u, 0u}, tot1[2] = {0u, 0u};

    auto flush = [&]() {
        __syncthreads();   // every wave is done with the word buffer
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int s = 0; s < HALF; ++s) lds[wv][s][lane] = acc[h * HALF + s];
            wave_sync();
            const int sl = lane & (HALF - 1), j0 = (lane >> 5) * HALF;
            for (int l = j0; l < j0 + HALF; ++l) {
                const uint32_t x = lds[wv][sl][l];
                totR[h] += x & 63u;
                tot0[h] += (x >> 6) & 4095u;
                tot1[h] += (x >> 18) & 4095u;
            }
            wave_sync();
        }
#pragma unroll
        for (int s = 0; s < NT; ++s) acc[s] = 0u;
        __syncthreads();   // transposes read before the next chunk's words land
    };

    int since = 0;
    for (uint32_t k00 = kb; k00 < ke; k00 += CPB * WAVE) {
        // this wave's Philox blocks of the phase's chunks, (chunk, block) pairs numbered 0..35: wv and
        // wv + 16, and 32 + wv / 2 for waves 1, 3, 5 and 7, which count the shorter (17-word) halves
        // (words of a chunk past the item's end are generated and never used)
        static_assert(CPB * NB == 2 * NWAVES + 4, "two blocks per wave and four more");
        const int nbb = (wv & 1) && wv < 8 ? 3 : 2;
        for (int i = 0; i < nbb; ++i) {
            const int bb = i < 2 ? wv + i * NWAVES : 2 * NWAVES + (wv >> 1);
            const int c = bb / NB, b = bb - c * NB;
            const u32x4 w = philox_block((uint32_t)b, k00 + (uint32_t)(c * WAVE + lane), key0, key1);
            uint32_t(*wc)[WAVE] = words + c * 4 * NB;
            wc[4 * b + 0][lane] = w.x;
            wc[4 * b + 1][lane] = w.y;
            wc[4 * b + 2][lane] = w.z;
            wc[4 * b + 3][lane] = w.w;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < CPB; ++c) {
            uint32_t yc[B2U];
#pragma unroll
            for (int u = 0; u < B2U; ++u) yc[u] = 0u;
            if (counting) {
                uint32_t(*wc)[WAVE] = words + c * 4 * NB;
#pragma unroll 6
                for (int j = 0; j < jn; ++j) {
                    const uint32_t x = wc[jw0 + j][lane];
#pragma unroll
                    for (int u = 0; u < B2U; ++u) yc[u] += (x < Tc[u]) ? 1u : 0u;
                }
            }
            cnt[c][wv][lane] = make_uint2(yc[0] | (yc[1] << 8) | (yc[2] << 16) | (yc[3] << 24),
                                          yc[4] | (yc[5] << 8) | (yc[6] << 16) | (yc[7] << 24));
        }
        __syncthreads();   // words consumed, counts shared: the next phase (or a flush) may overwrite the words
#pragma unroll
        for (int c = 0; c < CPB; ++c) {
        const uint32_t k0 = k00 + (uint32_t)(c * WAVE);
        if (!live || k0 >= ke) break;   // uniform: the item's range ends in the phase's first chunk
        const uint32_t k = k0 + (uint32_t)lane;
        const bool act = k < ke;
        {
            // the batch's row set (arm-0 counts) and column set (arm-1 counts), each the byte-wise
            // sum of its two halves
            const uint2 ra = cnt[c][rsrc][lane], rb = cnt[c][rsrc + 1][lane];
            const uint2 ca = cnt[c][csrc2][lane], cb = cnt[c][csrc2 + 1][lane];
            const uint2 rc = make_uint2(ra.x + rb.x, ra.y + rb.y);
            const uint2 cc = make_uint2(ca.x + cb.x, ca.y + cb.y);
            int y0[B2U], y1[B2V];
#pragma unroll
            for (int u = 0; u < B2U; ++u) y0[u] = (int)(((u < 4 ? rc.x : rc.y) >> (8 * (u & 3))) & 0xFFu);
#pragma unroll
            for (int v = 0; v < B2V; ++v) y1[v] = (int)(((v < 4 ? cc.x : cc.y) >> (8 * (v & 3))) & 0xFFu);
            if (KEYS) {
                // the block's records are padded to whole chunks: lanes past N store too (the
                // selection reads records k < N only)
                rbase[k] = make_uint4(rc.x, rc.y, cc.x, cc.y);
            }
            // reject indicator r = [y1 >= c(y0)] = med3(y1 - c + 1, 0, 1), added as r * packed
            // (24-bit multiply-add; no compare masks, so nothing is held in scalar registers)
            int cm[B2U];
            uint32_t P0[B2U], P1[B2V];
#pragma unroll
            for (int u = 0; u < B2U; ++u) {
                cm[u] = (act ? s_cut[y0[u]] : 64) - 1;
                P0[u] = 1u | ((uint32_t)y0[u] << 6);
            }
#pragma unroll
            for (int v = 0; v < B2V; ++v) P1[v] = (uint32_t)y1[v] << 18;
#pragma unroll
            for (int u = 0; u < B2U; ++u)
#pragma unroll
                for (int v = 0; v < B2V; ++v) {
                    const uint32_t r = (uint32_t)min(max(y1[v] - cm[u], 0), 1);
                    acc[u * B2V + v] += __umul24(r, P0[u] + P1[v]);
                }
        }
        }
        since += CPB;
        if (since > 63 - CPB) {   // at most 63 simulations per lane between flushes
            flush();
            since = 0;
        }
    }
    flush();
    if (!live) return;
#pragma unroll
    for (int h = 0; h < 2; ++h) {   // combine the two lane halves of each slot
        totR[h] += __shfl_xor(totR[h], HALF);
        tot0[h] += __shfl_xor(tot0[h], HALF);
        tot1[h] += __shfl_xor(tot1[h], HALF);
    }
    if (lane >= HALF) return;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int32_t tile = B->tile[h * HALF + lane];
        if (tile >= 0) {
            atomicAdd(&R[tile], totR[h]);
            atomicAdd(&sumT[2 * (int64_t)tile], (unsigned long long)tot0[h]);
            atomicAdd(&sumT[2 * (int64_t)tile + 1], (unsigned long long)tot1[h]);
        }
    }
}


// ------------------------------------------------------------------------------------
// z-test: X = theta + Z, Z from words 0 and 1 by Box-Muller in float32,
// u = ((word >> 9) + 1/2) 2^-23.  Reject X > cut; score term X - theta = Z; key S = -X.
// Score sums are carried in 64-bit fixed point (2^-32) so the cross-wave sum is exact.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ float unit23(uint32_t w) {
    return ((float)(w >> 9) + 0.5f) * (1.0f / 8388608.0f);
}

template <bool KEYS>
__global__ __launch_bounds__(WG) void k_ztest1(const Blk1 *__restrict__ blocks,
                                               const WorkItem *__restrict__ items, int64_t n_items,
                                               uint32_t key0, uint32_t key1, float cut,
                                               uint32_t *__restrict__ R,
                                               unsigned long long *__restrict__ sumZfx,
                                               float *__restrict__ keys) {
    constexpr int NT = B1T;
    __shared__ uint32_t xbuf[WG / WAVE][NT][WAVE + 1];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t it = (int64_t)blockIdx.x * (WG / WAVE) + wv;
    if (it >= n_items) return;
    const WorkItem W = items[it];
    const Blk1 *__restrict__ B = blocks + W.blk;
    const uint32_t n_sims = (uint32_t)B->n_sims;
    const int64_t key_base = B->key_base;

    uint32_t accR[NT];
    float accZ[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        accR[s] = 0u;
        accZ[s] = 0.0f;
    }
    uint32_t totR = 0u;
    long long totZ = 0;

    auto flush = [&]() {
#pragma unroll
        for (int s = 0; s < NT; ++s) xbuf[wv][s][lane] = accR[s];
        wave_sync();
        for (int l = 0; l < WAVE; ++l) totR += xbuf[wv][lane][l];
        wave_sync();
#pragma unroll
        for (int s = 0; s < NT; ++s) xbuf[wv][s][lane] = __float_as_uint(accZ[s]);
        wave_sync();
        for (int l = 0; l < WAVE; ++l)
            totZ += (long long)__double2ll_rn((double)__uint_as_float(xbuf[wv][lane][l]) * 4294967296.0);
        wave_sync();
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            accR[s] = 0u;
            accZ[s] = 0.0f;
        }
    };

    int since = 0;
    for (uint32_t k0 = W.k_begin; k0 < W.k_end; k0 += WAVE) {
        const uint32_t k = k0 + (uint32_t)lane;
        const bool act = k < W.k_end;
        const u32x4 w = philox_block(0u, k, key0, key1);
        const float u0 = unit23(w.x), u1 = unit23(w.y);
        const float Z = sqrtf(-2.0f * logf(u0)) * cospif(2.0f * u1);
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            const float X = B->theta[s] + Z;
            const bool r = act && (X > cut);
            accR[s] += r ? 1u : 0u;
            accZ[s] += r ? Z : 0.0f;
            if (KEYS && act && B->tile[s] >= 0) keys[key_base + (int64_t)s * n_sims + k] = -X;
        }
        if (++since == 16) {
            flush();
            since = 0;
        }
    }
    flush();
    const int32_t tile = B->tile[lane];
    if (tile >= 0) {
        atomicAdd(&R[tile], totR);
        atomicAdd(&sumZfx[tile], (unsigned long long)totZ);
    }
}

// ------------------------------------------------------------------------------------
// The plain forward-only path: one launch per tile, one simulation per thread, the tile's
// own thresholds, no sharing across tiles, rejection count only.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_binom2_plain(uint32_t T0, uint32_t T1, uint32_t n_sims,
                                                     uint32_t key0, uint32_t key1,
                                                     const int32_t *__restrict__ cut_tbl,
                                                     uint32_t *__restrict__ R_tile) {
    constexpr int NW = 2 * NP35;
    constexpr int NB = (NW + 3) / 4;
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    const uint32_t k = blockIdx.x * WG + threadIdx.x;
    uint32_t r = 0u;
    if (k < n_sims) {
        int y0 = 0, y1 = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const u32x4 w = philox_block((uint32_t)b, k, key0, key1);
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const int widx = 4 * b + l;
                const uint32_t x = u32x4_get(w, l);
                if (widx < NP35)
                    y0 += (x < T0) ? 1 : 0;
                else if (widx < NW)
                    y1 += (x < T1) ? 1 : 0;
            }
        }
        r = (y1 >= cut_tbl[y0]) ? 1u : 0u;
    }
    const unsigned long long m = __ballot(r);
    if ((threadIdx.x & (WAVE - 1)) == 0) atomicAdd(&s_cnt, (uint32_t)__popcll(m));
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(R_tile, s_cnt);
}

__global__ __launch_bounds__(WG) void k_ztest1_plain(float theta, float cut, uint32_t n_sims,
                                                     uint32_t key0, uint32_t key1,
                                                     uint32_t *__restrict__ R_tile) {
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    const uint32_t k = blockIdx.x * WG + threadIdx.x;
    uint32_t r = 0u;
    if (k < n_sims) {
        const u32x4 w = philox_block(0u, k, key0, key1);
        const float Z = sqrtf(-2.0f * logf(unit23(w.x))) * cospif(2.0f * unit23(w.y));
        r = (theta + Z > cut) ? 1u : 0u;
    }
    const unsigned long long m = __ballot(r);
    if ((threadIdx.x & (WAVE - 1)) == 0) atomicAdd(&s_cnt, (uint32_t)__popcll(m));
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(R_tile, s_cnt);
}

// ------------------------------------------------------------------------------ launchers
hipError_t launch_binom2(const Platten &P, uint64_t seed, uint32_t *R, unsigned long long *sumT,
                         uint4 *keys, hipStream_t st) {
    const int64_t grid = P.n_gitems;
    if (grid <= 0) return hipSuccess;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (keys)
        hipLaunchKernelGGL(k_binom2<true>, dim3((uint32_t)grid), dim3(WG2), 0, st,
                           (const Blk2 *)P.d_blocks, P.d_sqitems, P.n_gitems, k0, k1, P.d_cut_tbl, R,
                           sumT, keys);
    else
        hipLaunchKernelGGL(k_binom2<false>, dim3((uint32_t)grid), dim3(WG2), 0, st,
                           (const Blk2 *)P.d_blocks, P.d_sqitems, P.n_gitems, k0, k1, P.d_cut_tbl, R,
                           sumT, keys);
    return hipGetLastError();
}

hipError_t launch_ztest1(const Platten &P, uint64_t seed, uint32_t *R, unsigned long long *sumZfx,
                         float *keys, hipStream_t st) {
    const int64_t grid = (P.n_items + (WG / WAVE) - 1) / (WG / WAVE);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const float cut = (float)P.design.cut;
    if (keys)
        hipLaunchKernelGGL(k_ztest1<true>, dim3((uint32_t)grid), dim3(WG), 0, st,
                           (const Blk1 *)P.d_blocks, P.d_items, P.n_items, k0, k1, cut, R, sumZfx,
                           keys);
    else
        hipLaunchKernelGGL(k_ztest1<false>, dim3((uint32_t)grid), dim3(WG), 0, st,
                           (const Blk1 *)P.d_blocks, P.d_items, P.n_items, k0, k1, cut, R, sumZfx,
                           keys);
    return hipGetLastError();
}

hipError_t launch_plain_tile(const Platten &P, uint64_t seed, int64_t t, uint32_t T0, uint32_t T1,
                             uint32_t *R_tile, hipStream_t st) {
    const uint32_t N = (uint32_t)P.tile_N[t];
    const uint32_t grid = (N + WG - 1) / WG;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (P.design.kind == CSE_ZTEST1)
        hipLaunchKernelGGL(k_ztest1_plain, dim3(grid), dim3(WG), 0, st, (float)P.tile_theta[t],
                           (float)P.design.cut, N, k0, k1, R_tile);
    else
        hipLaunchKernelGGL(k_binom2_plain, dim3(grid), dim3(WG), 0, st, T0, T1, N, k0, k1,
                           P.d_cut_tbl, R_tile);
    return hipGetLastError();
}

}  // namespace cse
