// k_hier4.hip -- four Bernoulli arms (arm 0 control) under the hierarchical model of the
// basket case study (Section 10.1): theta_i | mu, s2 ~ N(mu, s2), mu ~ N(-1.34, 100),
// s2 ~ InvGamma(0.0005, 0.000005); statistic of treatment arm i: P(p_i > p_0 | y).
//
// Posterior table (one thread per outcome y in {0..n}^4), float64, by the Laplace node mixture
// of hier_post.hpp; the statistic 1 - P_i is summed directly as sum_j pi_j Phi(-z_j).
// The table holds float32 (1 - P_1, 1 - P_2, 1 - P_3, 0) per outcome, index ((y0 m + y1) m + y2) m + y3.
#include <math.h>

#include "cse_internal.h"
#include "fp64_math.hpp"
#include "hier_post.hpp"
#include "kernels.h"
#include "philox.hpp"

namespace cse {

__global__ __launch_bounds__(128) void k_hier4_table(int n, int64_t n_out, float4 *__restrict__ tbl,
                                                     const HierNode *__restrict__ nodes) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_out) return;
    const int m = n + 1;
    int y[4];
    {
        int64_t v = idx;
        for (int a = 3; a >= 0; --a) {
            y[a] = (int)(v % m);
            v /= m;
        }
    }
    const double nv[4] = {(double)n, (double)n, (double)n, (double)n};
    HierSummary s;
    hier_posterior<false, false>(y, nv, nodes, s);
    float4 o;
    o.x = (float)s.Sc[0];
    o.y = (float)s.Sc[1];
    o.z = (float)s.Sc[2];
    o.w = 0.0f;
    tbl[idx] = o;
}

// Basket design table: float32 (1 - P_0, .., 1 - P_3) per outcome, P_a = P(p_a > p_0a | y).
struct Theta0 {
    double v[4];
};
__global__ __launch_bounds__(128) void k_basket_table(int n, int64_t n_out, Theta0 t0, float4 *__restrict__ tbl,
                                                      const HierNode *__restrict__ nodes) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_out) return;
    const int m = n + 1;
    int y[4];
    {
        int64_t v = idx;
        for (int a = 3; a >= 0; --a) {
            y[a] = (int)(v % m);
            v /= m;
        }
    }
    double Sc[4];
    basket_posterior(y, (double)n, t0.v, nodes, Sc);
    tbl[idx] = make_float4((float)Sc[0], (float)Sc[1], (float)Sc[2], (float)Sc[3]);
}

hipError_t launch_basket_table(int n, const double *theta0, float4 *tbl, const HierNode *nodes, hipStream_t st) {
    const int64_t m = n + 1;
    const int64_t n_out = m * m * m * m;
    Theta0 t0;
    for (int a = 0; a < 4; ++a) t0.v[a] = theta0[a];
    hipLaunchKernelGGL(k_basket_table, dim3((uint32_t)((n_out + 127) / 128)), dim3(128), 0, st, n, n_out, t0, tbl,
                       nodes);
    return hipGetLastError();
}

// Rejection mask of every outcome at the design's cut (bit a-1 for treatment arm a of the
// 4-arm design, bit a for arm a of the basket design): the forward pass gathers this byte
// instead of the float4 row; the comparison is the one the keyed pass makes.
__global__ void k_h4_mask(const float4 *__restrict__ tbl, int64_t n, float cut, int nbits, uint8_t *__restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 q = tbl[i];
    uint32_t m = (q.x < cut ? 1u : 0u) | (q.y < cut ? 2u : 0u) | (q.z < cut ? 4u : 0u);
    if (nbits == 4 && q.w < cut) m |= 8u;
    mask[i] = (uint8_t)m;
}

hipError_t launch_h4_mask(const float4 *tbl, int64_t n, float cut, int nbits, uint8_t *mask, hipStream_t st) {
    hipLaunchKernelGGL(k_h4_mask, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, tbl, n, cut, nbits, mask);
    return hipGetLastError();
}

hipError_t launch_hier4_table(int n, float4 *tbl, const HierNode *nodes, hipStream_t st) {
    const int64_t m = n + 1;
    const int64_t n_out = m * m * m * m;
    hipLaunchKernelGGL(k_hier4_table, dim3((uint32_t)((n_out + 127) / 128)), dim3(128), 0, st, n, n_out, tbl,
                       nodes);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Fused simulation, 4 arms x 35 patients (words a*35 .. a*35+34 for arm a: 35 Philox blocks).
// The four waves of a workgroup run four box batches over the same simulations and share each
// chunk's 140 words through LDS.  Per (simulation, box slot): one 16-byte gather of
// (1 - P_1, 1 - P_2, 1 - P_3) at the outcome y; the design rejects treatment arm i when
// 1 - P_i < cut, giving a 3-bit mask m; configuration b's FWER event is m & b != 0.  Per box the
// lanes count each mask value (7 packed 2-bit counters per slot, two slots per word, exact for
// 3 simulations per lane between flushes, which transpose the counters through the word
// buffer), so R_b = sum_{m & b != 0} count[m] for every b of the box.  LDS is the 35 KB word
// buffer and the score rows, so four workgroups fit on a CU.
// Calibration keys: S_b = min_{i in b} (1 - P_i) per (simulation, tile), float32.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync4() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// BASKET: the basket design (four hypotheses, arm a <-> bit a, q.w used): every slot holds one
// piece with a single configuration b, so each lane counts that configuration's events in one
// 16-bit field per slot (two slots per word, flushed every 4,096 chunks).
// SCORE: also the score sums of every tile, sum over its rejecting simulations of the arm counts
// y_a (the sufficient statistic, Example 1), as packed pairs (y0 | y1 << 16, y2 | y3 << 16),
// added to the tile's row in LDS with LDS atomics.  4-arm lanes add their own pairs (rejections
// are rare at that design's cut).  Basket slots, where most simulations of a piece may reject, do
// so only when a few lanes reject; otherwise the pairs are first summed over each 16-lane row by
// DPP shifts and the four row totals are added (atomics of many lanes to one LDS word
// serialise).  At most 64 * 35 per row and
// chunk, so the 16-bit fields hold 15 chunks; the rows are added to the 64-bit tile sums in global
// memory at every flush.  Rows past H4_SROWS (rare batches with many cut boxes) add to global
// memory directly.
constexpr int H4_SROWS = 128;
constexpr int H4_FEW = 4;   // at most this many rejecting lanes: atomics straight from the lanes

// Inclusive scan over the 16 lanes of each DPP row by row shifts of 1, 2, 4, 8 (shifted-in lanes
// read 0): lane 15 of each row ends with the row's total.  Call with every lane active.
__device__ __forceinline__ uint32_t row16_sum(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);   // row_shr:8
    return v;
}
constexpr uint64_t H4_REJ = 0xFEFCFAF0EECCAA00ull;   // byte m: configurations b (bits 1..7) with m & b != 0

// Bracketed keys (KEYS = 2; blocks of at most H4_BROWS key rows): per tile the bracket (lo, hi)
// from the pilot; the pass counts the keys below lo (per wave and key row in LDS, added to the
// tile at the end of the item) and keeps
// those in [lo, hi] in the tile's region of the item's range (caps slots; the count goes on past
// caps, which sends the tile to the exact path).
struct H4Brk {
    const float2 *brk;
    uint32_t *below;
    uint32_t *cnt;     // per tile [1 + maxs]: [0] the pilot's candidates, [1 + s] item range s
    float *cand;       // per tile [tot]: H4_PCAP pilot slots, then caps per item range
    int64_t tot;
    int32_t maxs, caps;
    uint32_t k_lo;     // first simulation of the pass (the pilot holds the ones before)
};
template <int KEYS, bool BASKET, bool SCORE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_hier4(const Blk4 *__restrict__ blocks,
                                              const GroupItem *__restrict__ items, int64_t n_items,
                                              uint32_t key0, uint32_t key1,
                                              const float4 *__restrict__ tbl, const uint8_t *__restrict__ mtbl,
                                              float cut, uint32_t *__restrict__ R,
                                              unsigned long long *__restrict__ sumT, float *__restrict__ keys,
                                              H4Brk hb) {
    static_assert(KEYS != 2 || !BASKET, "bracketed keys serve the 4-arm design");
    constexpr int NP = NP35;
    constexpr int NW = 4 * NP;
    constexpr int NB = NW / 4;   // 35 Philox blocks
    constexpr int NBH = (NB + 1) / 2;   // blocks of the first half (18: words 0..71), then 17 (words 72..139)
    constexpr int NWH = 4 * NBH;        // words held at once
    constexpr int NWAVES = WG / WAVE;
    constexpr int M1 = NP + 1;
    constexpr int FLUSH_EVERY = 15;        // score rows: 16-bit fields hold 15 chunks
    // Half of the chunk's Philox words at a time; between chunks the same memory holds the
    // counter transposes (per wave 16 x (64 + 1) words, padded against bank conflicts).
    __shared__ uint32_t words[NWH][WAVE];
    __shared__ uint2 ysum[SCORE ? NWAVES : 1][SCORE ? H4_SROWS : 1];   // per wave and key row: packed y sums
    // bracketed keys: per wave and key row, the tile's bracket (lo, hi as float bits), the keys
    // below it and the candidates kept in this item; and the row's tile
    __shared__ uint4 rcnt[KEYS == 2 ? NWAVES : 1][KEYS == 2 ? H4_BROWS : 1];
    __shared__ int32_t rtile[KEYS == 2 ? NWAVES : 1][KEYS == 2 ? H4_BROWS : 1];

    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t it = blockIdx.x;
    if (it >= n_items) return;
    const GroupItem *__restrict__ G = items + it;
    const int32_t blk = G->blk[wv];   // read in place: a register copy indexed by wv would go to scratch
    const bool live = blk >= 0;
    const Blk4 *__restrict__ B = blocks + (live ? blk : G->blk[0]);
    const uint32_t kb = KEYS == 2 ? max(G->k_begin, hb.k_lo) : G->k_begin, ke = G->k_end;
    uint32_t T0[B4N0], T1[B4N1], T2[B4N2], T3[B4N3];
#pragma unroll
    for (int u = 0; u < B4N0; ++u) T0[u] = B->T0[u];
#pragma unroll
    for (int u = 0; u < B4N1; ++u) T1[u] = B->T1[u];
#pragma unroll
    for (int u = 0; u < B4N2; ++u) T2[u] = B->T2[u];
#pragma unroll
    for (int u = 0; u < B4N3; ++u) T3[u] = B->T3[u];
    const int32_t n_rows = B->n_rows;
    float *__restrict__ kbase = keys + (KEYS == 1 ? B->key_base : 0);
    const int32_t slice = G->slice;
    if (KEYS == 2 && live) {
        static_assert(B4S == WAVE, "one lane per slot");
        const int32_t r0 = B->row0[lane];
        if (r0 >= 0) {
            const int nq = __popc(B->bmask[lane]);
            for (int q = 0; q < nq && r0 + q < H4_BROWS; ++q) {
                const int32_t t = B->tile0[lane] + q;
                const float2 br = hb.brk[t];
                rtile[wv][r0 + q] = t;
                rcnt[wv][r0 + q] = make_uint4(__float_as_uint(br.x), __float_as_uint(br.y), 0u, 0u);
            }
        }
        wave_sync4();
    }
    // one key of a bracketed row (every lane of the wave calls): below the bracket it is counted,
    // inside it kept at the next free slot of the tile's region for this item range
    // (the plattens that take this pass have at most H4_BROWS key rows per block)
    auto take_key = [&](bool act_key, int32_t row, int32_t tile, float sb) {
        const uint4 v = rcnt[wv][row];   // bracket and counts (one LDS read, the same address in every lane)
        const float lo = __uint_as_float(v.x), hi = __uint_as_float(v.y);
        const bool bl = act_key && sb < lo;
        const bool in = act_key && sb >= lo && sb <= hi;
        const unsigned long long mb = __ballot(bl), mi = __ballot(in);
        if (!(mb | mi)) return;   // uniform
        if (lane == 0) {
            rcnt[wv][row].z = v.z + (uint32_t)__popcll(mb);
            rcnt[wv][row].w = v.w + (uint32_t)__popcll(mi);
        }
        if (in) {
            const uint32_t pos = v.w + (uint32_t)__popcll(mi & ((1ull << lane) - 1ull));
            if (pos < (uint32_t)hb.caps) hb.cand[(int64_t)tile * hb.tot + H4_PCAP + (int64_t)slice * hb.caps + pos] = sb;
        }
    };

    if (SCORE)
        for (int r = lane; r < H4_SROWS; r += WAVE) ysum[wv][r] = make_uint2(0u, 0u);
    // packed count pairs into a tile's row (LDS) or, past the LDS rows, its 64-bit sums
    auto add_pairs = [&](int32_t row, int32_t tile, uint32_t lo, uint32_t hi) {
        if (row < H4_SROWS) {
            atomicAdd(&ysum[wv][row].x, lo);
            atomicAdd(&ysum[wv][row].y, hi);
        } else {
            atomicAdd(&sumT[4 * (int64_t)tile + 0], (unsigned long long)(lo & 0xFFFFu));
            atomicAdd(&sumT[4 * (int64_t)tile + 1], (unsigned long long)(lo >> 16));
            atomicAdd(&sumT[4 * (int64_t)tile + 2], (unsigned long long)(hi & 0xFFFFu));
            atomicAdd(&sumT[4 * (int64_t)tile + 3], (unsigned long long)(hi >> 16));
        }
    };
    // one lane's counts (y0, y1, y2, y3) into a tile's sums
    auto add_counts = [&](int32_t row, int32_t tile, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
        if (row < H4_SROWS) {
            atomicAdd(&ysum[wv][row].x, a | (b << 16));
            atomicAdd(&ysum[wv][row].y, c | (d << 16));
        } else {
            atomicAdd(&sumT[4 * (int64_t)tile + 0], (unsigned long long)a);
            atomicAdd(&sumT[4 * (int64_t)tile + 1], (unsigned long long)b);
            atomicAdd(&sumT[4 * (int64_t)tile + 2], (unsigned long long)c);
            atomicAdd(&sumT[4 * (int64_t)tile + 3], (unsigned long long)d);
        }
    };
    // the counts of the lanes whose simulation rejects (ev) into the tile's sums; every lane calls
    auto add_score = [&](bool ev, int32_t row, int32_t tile, uint32_t lo, uint32_t hi) {
        const unsigned long long bal = __ballot(ev);
        if (!bal) return;
        if (__popcll(bal) <= H4_FEW) {
            if (ev) add_pairs(row, tile, lo, hi);
            return;
        }
        const uint32_t a = row16_sum(ev ? lo : 0u), b = row16_sum(ev ? hi : 0u);
        if ((lane & 15) == 15 && (a | b)) add_pairs(row, tile, a, b);
    };
    // the LDS rows into the tiles' 64-bit sums (lanes take a slot's rows), then cleared
    auto flush_scores = [&]() {
        wave_sync4();
        for (int s = 0; s < B4S; ++s) {
            const int32_t r0 = B->row0[s];
            if (r0 < 0) continue;   // uniform
            const int nq = BASKET ? 1 : __popc(B->bmask[s]);
            const int r = r0 + lane;
            if (lane < nq && r < H4_SROWS) {
                const uint2 v = ysum[wv][r];
                if (v.x | v.y) {
                    const int64_t t = (int64_t)B->tile0[s] + lane;
                    atomicAdd(&sumT[4 * t + 0], (unsigned long long)(v.x & 0xFFFFu));
                    atomicAdd(&sumT[4 * t + 1], (unsigned long long)(v.x >> 16));
                    atomicAdd(&sumT[4 * t + 2], (unsigned long long)(v.y & 0xFFFFu));
                    atomicAdd(&sumT[4 * t + 3], (unsigned long long)(v.y >> 16));
                    ysum[wv][r] = make_uint2(0u, 0u);
                }
            }
        }
        wave_sync4();
    };

    // One word per pair of slots (2p, 2p + 1).  4-arm: seven 2-bit fields per slot, field m - 1 of
    // slot 2p + h at bit 14 h + 2 (m - 1), counting the simulations with rejection mask m (at most
    // ACC_EVERY = 3 per lane between flushes); basket: a 16-bit count per slot at bit 16 h.
    // Half the registers of one word per slot, which leaves room for a whole group's table rows.
    constexpr int NACC = B4S / 2;
    constexpr int ACC_EVERY = BASKET ? 4096 : 3;
    constexpr int TRW = NACC / 2;   // counter words per flush half
    static_assert(NWAVES * TRW * (WAVE + 1) <= NWH * WAVE, "flush transposes must fit in the word buffer");
    uint32_t(*tr)[TRW][WAVE + 1] = reinterpret_cast<uint32_t(*)[TRW][WAVE + 1]>(&words[0][0]);
    uint32_t acc[NACC];
#pragma unroll
    for (int p = 0; p < NACC; ++p) acc[p] = 0u;
    // the counters of the chunks since the last flush into R: the wave transposes the words
    // through the word buffer, lanes l and l + 32 sum word l over their halves of the simulations
    // (byte-wise: four fields at a time, at most 3 x 64 per byte), and lane l adds the per-
    // configuration totals of slots 2l and 2l + 1
    auto flush = [&]() {
        __syncthreads();   // the word buffer is free: every wave has finished counting
#pragma unroll
        for (int h = 0; h < 2; ++h) {   // counter words 16 h .. 16 h + 15 (slots 32 h .. 32 h + 31)
#pragma unroll
            for (int p = 0; p < TRW; ++p) tr[wv][p][lane] = acc[h * TRW + p];
            wave_sync4();
            const int pw = lane & (TRW - 1), j0 = (lane / TRW) * (WAVE / 4);
            uint32_t A[4] = {0u, 0u, 0u, 0u};
            for (int j = j0; j < j0 + WAVE / 4; ++j) {
                const uint32_t x = tr[wv][pw][j];
                if (BASKET) {
                    A[0] += x & 0xFFFFu;
                    A[1] += x >> 16;
                    continue;
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) A[c] += (x >> (2 * c)) & 0x03030303u;
            }
            wave_sync4();
#pragma unroll
            for (int c = 0; c < 4; ++c) {   // the four lane groups' sums (at most 3 x 64 per byte)
                A[c] += __shfl_xor(A[c], TRW);
                A[c] += __shfl_xor(A[c], 2 * TRW);
            }
            if (live && lane < TRW) {
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int s = 2 * (h * TRW + pw) + hh;
                    const int32_t t0 = B->tile0[s];
                    if (t0 < 0) continue;
                    if (BASKET) {
                        if (A[hh]) atomicAdd(&R[t0], A[hh]);
                        continue;
                    }
                    uint32_t cnt[8];
#pragma unroll
                    for (int m = 1; m <= 7; ++m) {
                        const int f = 7 * hh + m - 1;   // field f: byte f / 4 of class f % 4
                        cnt[m] = (A[f % 4] >> (8 * (f / 4))) & 0xFFu;
                    }
                    const uint32_t bm = B->bmask[s];
                    int q = 0;
#pragma unroll
                    for (int b = 1; b <= 7; ++b) {
                        if (!(bm & (1u << b))) continue;
                        uint32_t r = 0u;
#pragma unroll
                        for (int m = 1; m <= 7; ++m)
                            if (m & b) r += cnt[m];
                        if (r) atomicAdd(&R[t0 + q], r);
                        ++q;
                    }
                }
            }
            wave_sync4();   // this half's transposes are read before the next half's are written
        }
#pragma unroll
        for (int p = 0; p < NACC; ++p) acc[p] = 0u;
        __syncthreads();   // transposes read before the next chunk's words overwrite them
    };

    int since = 0, since_acc = 0;
    for (uint32_t k0 = kb; k0 < ke; k0 += WAVE) {
        const uint32_t k = k0 + (uint32_t)lane;
        const bool act = k < ke;
        // the words in two halves (LDS for half of them at a time): blocks 0..17 give arms 0
        // and 1 and the first two words of arm 2, blocks 18..34 the rest of arm 2 and arm 3
        int y0[B4N0], y1[B4N1], y2[B4N2], y3[B4N3];
#pragma unroll
        for (int u = 0; u < B4N0; ++u) y0[u] = 0;
#pragma unroll
        for (int u = 0; u < B4N1; ++u) y1[u] = 0;
#pragma unroll
        for (int u = 0; u < B4N2; ++u) y2[u] = 0;
#pragma unroll
        for (int u = 0; u < B4N3; ++u) y3[u] = 0;
        for (int b = wv; b < NBH; b += NWAVES) {
            const u32x4 w = philox_block((uint32_t)b, k, key0, key1);
            words[4 * b + 0][lane] = w.x;
            words[4 * b + 1][lane] = w.y;
            words[4 * b + 2][lane] = w.z;
            words[4 * b + 3][lane] = w.w;
        }
        __syncthreads();
        if (live) {
#pragma unroll 7
            for (int j = 0; j < NP; ++j) {
                const uint32_t x = words[j][lane];
#pragma unroll
                for (int u = 0; u < B4N0; ++u) y0[u] += (x < T0[u]) ? 1 : 0;
            }
#pragma unroll 7
            for (int j = NP; j < 2 * NP; ++j) {
                const uint32_t x = words[j][lane];
#pragma unroll
                for (int u = 0; u < B4N1; ++u) y1[u] += (x < T1[u]) ? 1 : 0;
            }
#pragma unroll
            for (int j = 2 * NP; j < NWH; ++j) {
                const uint32_t x = words[j][lane];
#pragma unroll
                for (int u = 0; u < B4N2; ++u) y2[u] += (x < T2[u]) ? 1 : 0;
            }
        }
        __syncthreads();   // the first half is counted: its memory takes the second
        for (int b = NBH + wv; b < NB; b += NWAVES) {
            const u32x4 w = philox_block((uint32_t)b, k, key0, key1);
            words[4 * (b - NBH) + 0][lane] = w.x;
            words[4 * (b - NBH) + 1][lane] = w.y;
            words[4 * (b - NBH) + 2][lane] = w.z;
            words[4 * (b - NBH) + 3][lane] = w.w;
        }
        __syncthreads();
        if (live) {
#pragma unroll 11
            for (int j = NWH; j < 3 * NP; ++j) {
                const uint32_t x = words[j - NWH][lane];
#pragma unroll
                for (int u = 0; u < B4N2; ++u) y2[u] += (x < T2[u]) ? 1 : 0;
            }
#pragma unroll 7
            for (int j = 3 * NP; j < 4 * NP; ++j) {
                const uint32_t x = words[j - NWH][lane];
#pragma unroll
                for (int u = 0; u < B4N3; ++u) y3[u] += (x < T3[u]) ? 1 : 0;
            }
        }
        __syncthreads();
        if (live) {
            float *__restrict__ kc = kbase + (size_t)(k0 / WAVE) * n_rows * WAVE + lane;
            // Neighbouring thresholds of an arm often give a simulation the same count, and then
            // two slots share the outcome.  The slots of one u0 and GU1 consecutive u1 form a
            // group (16 slots; 8 in the keyed variants, whose rows take three registers each and
            // which run 5 waves per SIMD): its gathers are issued first, skipping a slot whose
            // outcome equals that of the slot at the previous u1 (same group), u3 or u2 (fewer
            // gathers are fewer L2 requests, the table being read at random rows), then one
            // wait, then the slots are evaluated and their keys stored.  Vector memory counts
            // loads and stores together, so a gather used right after the previous slot's key
            // stores would also wait for those stores.
            constexpr int S2 = B4N3, S1 = B4N2 * B4N3;
            constexpr int GU1 = KEYS == 2 ? 1 : (KEYS ? 2 : B4N1);   // u1 values per group (keyed: fewer rows in registers)
            constexpr int G = GU1 * S1;
#pragma unroll
            for (int ug = 0; ug < B4N0 * (B4N1 / GU1); ++ug) {
                const int u0 = ug / (B4N1 / GU1), u1b = (ug % (B4N1 / GU1)) * GU1;
                float4 qs[G];
                uint32_t ms[G];
                // whether slot i of the group repeats the outcome of the slot at u1 - 1 (same group),
                // u3 - 1 or u2 - 1
                auto repeats = [&](int i, bool &r1, bool &r3, bool &r2) {
                    const int i1 = i / S1, u1 = u1b + i1, u2 = (i / S2) % B4N2, u3 = i % S2;
                    const int s = (u0 * B4N1 + u1) * S1 + u2 * S2 + u3;
                    r1 = i1 > 0 && B->row0[i1 > 0 ? s - S1 : s] >= 0 && y1[u1] == y1[u1 > 0 ? u1 - 1 : 0];
                    r3 = u3 > 0 && B->row0[u3 > 0 ? s - 1 : s] >= 0 && y3[u3] == y3[u3 > 0 ? u3 - 1 : 0];
                    r2 = u2 > 0 && B->row0[u2 > 0 ? s - S2 : s] >= 0 && y2[u2] == y2[u2 > 0 ? u2 - 1 : 0];
                };
#pragma unroll
                for (int i = 0; i < G; ++i) {
                    const int u1 = u1b + i / S1, u2 = (i / S2) % B4N2, u3 = i % S2;
                    const int s = (u0 * B4N1 + u1) * S1 + u2 * S2 + u3;
                    qs[i] = make_float4(0.f, 0.f, 0.f, 0.f);
                    ms[i] = 0u;
                    if (B->row0[s] < 0) continue;   // uniform: the slot holds no box
                    bool r1, r3, r2;
                    repeats(i, r1, r3, r2);
                    if (!(r1 || r2 || r3)) {
                        const int idx = ((y0[u0] * M1 + y1[u1]) * M1 + y2[u2]) * M1 + y3[u3];
                        if (KEYS) qs[i] = tbl[idx];
                        else ms[i] = (uint32_t)mtbl[idx];
                    }
                }
                // vmcnt 0, expcnt and lgkmcnt left alone: the group's rows are in registers
                __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
                for (int i = 0; i < G; ++i) {
                    const int u1 = u1b + i / S1, u2 = (i / S2) % B4N2, u3 = i % S2;
                    const int s = (u0 * B4N1 + u1) * S1 + u2 * S2 + u3;
                    const int32_t row0 = B->row0[s];
                    if (row0 < 0) continue;   // uniform
                    bool r1, r3, r2;
                    repeats(i, r1, r3, r2);
                    const int i1 = i >= S1 ? i - S1 : i, i3 = u3 > 0 ? i - 1 : i, i2 = u2 > 0 ? i - S2 : i;
                    // a repeat takes its source's row (resolved earlier in the group); selects
                    // between values, not between array elements (a select of addresses would keep
                    // the arrays out of registers)
                    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
                    uint32_t m;
                    if (KEYS) {
                        const float4 a1 = qs[i1], a3 = qs[i3], a2 = qs[i2], a0 = qs[i];
                        q.x = r1 ? a1.x : (r3 ? a3.x : (r2 ? a2.x : a0.x));
                        q.y = r1 ? a1.y : (r3 ? a3.y : (r2 ? a2.y : a0.y));
                        q.z = r1 ? a1.z : (r3 ? a3.z : (r2 ? a2.z : a0.z));
                        if (BASKET) q.w = r1 ? a1.w : (r3 ? a3.w : (r2 ? a2.w : a0.w));
                        qs[i] = q;
                        m = act ? ((q.x < cut ? 1u : 0u) | (q.y < cut ? 2u : 0u) | (q.z < cut ? 4u : 0u) |
                                   (BASKET && q.w < cut ? 8u : 0u))
                                : 0u;
                    } else {
                        const uint32_t mm = r1 ? ms[i1] : (r3 ? ms[i3] : (r2 ? ms[i2] : ms[i]));
                        ms[i] = mm;
                        m = act ? mm : 0u;
                    }
                            if (BASKET) {
                                const uint32_t b = (uint32_t)__builtin_ctz(B->bmask[s]);   // the slot's one b
                                acc[s >> 1] += (m & b) ? 1u << (16 * (s & 1)) : 0u;
                                if (SCORE)
                                    add_score((m & b) != 0u, row0, B->tile0[s], (uint32_t)(y0[u0] | (y1[u1] << 16)),
                                              (uint32_t)(y2[u2] | (y3[u3] << 16)));
                                if (KEYS) {
                                    float sb = INFINITY;
                                    if (b & 1u) sb = fminf(sb, q.x);
                                    if (b & 2u) sb = fminf(sb, q.y);
                                    if (b & 4u) sb = fminf(sb, q.z);
                                    if (b & 8u) sb = fminf(sb, q.w);
                                    kc[(size_t)row0 * WAVE] = sb;
                                }
                                continue;
                            }
                            acc[s >> 1] += m ? 1u << (14 * (s & 1) + 2 * (m - 1)) : 0u;
                            if (SCORE) {
                                // the box's configurations b whose event m & b != 0 happened: byte m of
                                // H4_REJ has bit b set when m & b != 0.  Rejections are rare at the 4-arm
                                // design's cut, so the lanes add their own counts.
                                const uint32_t bm = B->bmask[s];
                                uint32_t rej = (uint32_t)(H4_REJ >> (8u * m)) & bm;
                                while (rej) {
                                    const uint32_t b = (uint32_t)__builtin_ctz(rej);
                                    rej &= rej - 1u;
                                    const int q = __popc(bm & ((1u << b) - 1u));   // the tile's rank in the box
                                    add_counts(row0 + q, B->tile0[s] + q, (uint32_t)y0[u0], (uint32_t)y1[u1],
                                               (uint32_t)y2[u2], (uint32_t)y3[u3]);
                                }
                            }
                            if constexpr (KEYS == 1) {
                                const uint32_t bm = B->bmask[s];
                                int row = row0;
#pragma unroll
                                for (int b = 1; b <= 7; ++b) {
                                    if (!(bm & (1u << b))) continue;   // uniform
                                    float sb = INFINITY;
                                    if (b & 1) sb = fminf(sb, q.x);
                                    if (b & 2) sb = fminf(sb, q.y);
                                    if (b & 4) sb = fminf(sb, q.z);
                                    kc[(size_t)row * WAVE] = sb;
                                    ++row;
                                }
                            } else if constexpr (KEYS == 2) {
                                // a loop, not unrolled: seven copies of the bracket step per slot would
                                // keep the slot loop from unrolling (and its rows from registers)
                                uint32_t bm = B->bmask[s];
                                int row = row0;
#pragma unroll 1
                                while (bm) {   // uniform
                                    const uint32_t b = (uint32_t)__builtin_ctz(bm);
                                    bm &= bm - 1u;
                                    float sb = INFINITY;
                                    if (b & 1u) sb = fminf(sb, q.x);
                                    if (b & 2u) sb = fminf(sb, q.y);
                                    if (b & 4u) sb = fminf(sb, q.z);
                                    take_key(act, row, B->tile0[s] + (row - row0), sb);
                                    ++row;
                                }
                            }
                }
            }
        }
        if (++since_acc == ACC_EVERY) {
            flush();
            since_acc = 0;
        }
        if (SCORE && ++since == FLUSH_EVERY) {
            if (live) flush_scores();
            since = 0;
        }
    }
    flush();
    if (SCORE && live) flush_scores();
    if (KEYS == 2 && live) {   // this item's counts of the LDS rows into their tiles
        wave_sync4();
        const int nr = min(B->n_rows, H4_BROWS);
        for (int r = lane; r < nr; r += WAVE) {
            const uint4 v = rcnt[wv][r];
            const int32_t t = rtile[wv][r];
            if (v.z) atomicAdd(&hb.below[t], v.z);
            hb.cnt[(int64_t)t * (hb.maxs + 1) + 1 + slice] = v.w;
        }
    }
}

hipError_t launch_hier4(const Platten &P, uint64_t seed, uint32_t *R, unsigned long long *sumT, float *keys,
                        hipStream_t st, int pass) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const float cut = (float)P.design.cut;
    const bool basket = P.design.kind == CSE_BASKET4;
    H4Brk hb{P.d_h4brk, P.d_h4below, P.d_h4cnt, P.d_h4cand, P.h4_tot, P.h4_maxs, P.h4_caps, (uint32_t)H4_PILOT};
    const GroupItem *items = P.d_gitems;
    int64_t n_items = P.n_gitems;
    if (pass == H4_PASS_PILOT) {
        if (basket || !keys) return hipErrorInvalidValue;
        items = P.d_gitems_pilot;
        n_items = P.n_gitems_pilot;
    } else if (pass == H4_PASS_MAIN && (basket || !P.d_h4cand)) {
        return hipErrorInvalidValue;
    }
    if (n_items == 0) return hipSuccess;
#define CSE_H4_LAUNCH(K, BK, SC)                                                                                  \
    hipLaunchKernelGGL((k_hier4<K, BK, SC>), dim3((uint32_t)n_items), dim3(WG), 0, st, (const Blk4 *)P.d_blocks, \
                       items, n_items, k0, k1, P.d_h4tbl, P.d_h4mask, cut, R, sumT, keys, hb)
#define CSE_H4_SC(K, BK)            \
    if (sumT)                       \
        CSE_H4_LAUNCH(K, BK, true); \
    else                            \
        CSE_H4_LAUNCH(K, BK, false)
    if (pass == H4_PASS_MAIN) {
        CSE_H4_SC(2, false);
    } else if (keys && basket) {
        CSE_H4_SC(1, true);
    } else if (keys) {
        CSE_H4_SC(1, false);
    } else if (basket) {
        CSE_H4_SC(0, true);
    } else {
        CSE_H4_SC(0, false);
    }
#undef CSE_H4_SC
#undef CSE_H4_LAUNCH
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Plain forward path: one launch per tile (box centre, configuration b), one simulation per
// thread, each thread drawing its own 140 words; the baseline the fused kernel is timed against.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_hier4_plain(uint32_t T0, uint32_t T1, uint32_t T2, uint32_t T3,
                                                    uint32_t bmask, uint32_t n_sims, uint32_t key0,
                                                    uint32_t key1, const float4 *__restrict__ tbl,
                                                    float cut, uint32_t *__restrict__ R_tile) {
    constexpr int NP = NP35;
    constexpr int M1 = NP + 1;
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    const uint32_t k = blockIdx.x * WG + threadIdx.x;
    uint32_t r = 0u;
    if (k < n_sims) {
        int y[4] = {0, 0, 0, 0};
        const uint32_t T[4] = {T0, T1, T2, T3};
#pragma unroll
        for (int b = 0; b < NP; ++b) {   // 4 * 35 words = 35 blocks
            const u32x4 w = philox_block((uint32_t)b, k, key0, key1);
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const int widx = 4 * b + l;
                const int a = widx / NP;
                y[a] += (u32x4_get(w, l) < T[a]) ? 1 : 0;
            }
        }
        const float4 q = tbl[((y[0] * M1 + y[1]) * M1 + y[2]) * M1 + y[3]];
        float sb = INFINITY;
        if (bmask & 1u) sb = fminf(sb, q.x);
        if (bmask & 2u) sb = fminf(sb, q.y);
        if (bmask & 4u) sb = fminf(sb, q.z);
        if (bmask & 8u) sb = fminf(sb, q.w);   // basket design only (arm 3 is a hypothesis)
        r = (sb < cut) ? 1u : 0u;
    }
    const unsigned long long m = __ballot(r);
    if ((threadIdx.x & (WAVE - 1)) == 0) atomicAdd(&s_cnt, (uint32_t)__popcll(m));
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(R_tile, s_cnt);
}

hipError_t launch_hier4_plain(const Platten &P, uint64_t seed, int64_t t, uint32_t *R_tile, hipStream_t st) {
    const uint32_t N = (uint32_t)P.tile_N[t];
    const uint32_t grid = (N + WG - 1) / WG;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t *T = &P.tile_T[t * 4];
    hipLaunchKernelGGL(k_hier4_plain, dim3(grid), dim3(WG), 0, st, T[0], T[1], T[2], T[3],
                       (uint32_t)P.tile_cfg[t], N, k0, k1, P.d_h4tbl, (float)P.design.cut, R_tile);
    return hipGetLastError();
}

}  // namespace cse
