// k_select.hip -- the calibrated threshold of each tile, lambda*_i = S_(k_i), the k_i-th
// smallest statistic among the tile's N_i simulations (Section 7.1), the count of
// simulations strictly below it, and lambda* = min_i lambda*_i (Section 7.3).
// One workgroup per tile, counts in LDS.  Plus the small per-tile finishing kernels
// (score gradient, fixed-point conversion, zero fill).
#include <math.h>

#include <algorithm>

#include "cse_internal.h"
#include "kernels.h"
#include "philox.hpp"

namespace cse {

constexpr int SEL_WG = 256;

// Block-wide exclusive scan of one value per thread (SEL_WG threads), result in part[tid]:
// an inclusive scan within each wave by lane shuffles, then the totals of the waves before.
__device__ void block_exclusive_scan(uint32_t v, uint32_t *part) {
    __shared__ uint32_t wave_tot[SEL_WG / WAVE];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == WAVE - 1) wave_tot[w] = x;
    __syncthreads();
    uint32_t before = 0u;
    for (int i = 0; i < w; ++i) before += wave_tot[i];
    part[tid] = before + x - v;
    __syncthreads();   // wave_tot may be rewritten by the next call only after every wave read it
}

// ---- discrete statistic (2-arm design) ----
// The fused kernel stores one record per (simulation, batch): the success counts y0[u], y1[v] at
// the batch's 8 + 8 thresholds (Rec2), so tile (u, v)'s outcome of simulation j is
// y0[u] (n+1) + y1[v].  The statistic S = -z is a function of the outcome; outcomes sorted by S
// (S_order, ties grouped by S_group: the first position with equal S) give each outcome a
// position S_pos, and the k-th smallest S of a tile is the S of the first position whose
// cumulative count reaches k.
//
// Selection in three kernels:
//  * k_b2_bracket: per tile, the exact law of (y0, y1) under the simulated model (independent
//    Binomial(35, T/2^32) arms) gives a bracket [lo, hi] of positions (whole tie groups, found by
//    binary search over the groups) holding the k-th smallest S unless the count below lo reaches
//    k or the count up to hi stays below k, each a margin (5 by default, cse_platten_set_option)
//    of standard deviations of the count away.
//    As S does not increase with y1 for fixed y0, S < S(lo) iff y1 >= clo(y0) and S <= S(hi) iff
//    y1 >= chi(y0): the kernel also writes, per batch row u and count y0, the cut points clo, chi
//    of the row's 8 tiles as bytes (16 bytes);
//  * k_b2_select: one workgroup per batch reads the batch's records once.  Per simulation and
//    row, one LDS read of the row's cut bytes classifies its 8 tiles four at a time (byte-wise
//    compares of the record's packed y1 bytes): tiles below the bracket are counted in packed
//    byte counters per lane, and the rare tiles inside it look up the outcome's position and
//    add to an LDS histogram of the bracket; the k-th smallest is read off the histogram;
//  * k_b2_full: tiles whose k-th smallest fell outside the bracket, or whose bracket did not fit
//    the LDS histogram, are selected from a full 1,296-bin histogram of their records.
// Either way lambda*_i is the exact k-th smallest S and rej_at the exact count strictly below it.
constexpr int B2_N1 = NP35 + 1;            // outcomes per arm
constexpr int B2_NOUT = B2_N1 * B2_N1;     // 1,296 outcomes
constexpr int B2_HB = 4096;                // LDS histogram bins of one batch (16 KB)

__device__ __forceinline__ uint32_t rec_byte(uint32_t w, int b) { return (w >> (8 * b)) & 0xFFu; }
__device__ __forceinline__ uint32_t rec_outcome(const uint4 r, int s) {
    const int u = s >> 3, v = s & 7;
    const uint32_t y0 = rec_byte(u < 4 ? r.x : r.y, u & 3);
    const uint32_t y1 = rec_byte(v < 4 ? r.z : r.w, v & 3);
    return y0 * (uint32_t)B2_N1 + y1;
}

__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per batch, lane = slot.  Also resets the fallback list (before k_b2_select runs).
// Under the exact law, P(S < S_g) = sum_y0 P(y0) P(y1 >= cut_g(y0)) for each tie group g (S does
// not increase with y1), so each bracket end is a binary search over the tie groups with 36 terms
// per evaluation, and the cut bytes of the selection are the table rows of the two groups found.
__global__ __launch_bounds__(WAVE) void k_b2_bracket(const Blk2 *__restrict__ blocks, const int32_t *__restrict__ kk,
                                                     const int32_t *__restrict__ gstart,
                                                     const uint8_t *__restrict__ gcut, int n_groups,
                                                     int2 *__restrict__ br, uint4 *__restrict__ cut,
                                                     uint32_t *__restrict__ fb, float zmargin) {
    __shared__ float tail1[B2_N1 + 1][WAVE];   // P(y1 >= c) of each lane's tile, c = 0..36
    __shared__ uint8_t cb[B2U][B2_N1][16];     // per row and y0: clo of the 8 tiles, then chi
    const int lane = threadIdx.x;
    const Blk2 *__restrict__ B = blocks + blockIdx.x;
    if (blockIdx.x == 0 && lane == 0) fb[0] = 0u;
    const int32_t t = B->tile[lane];
    const int32_t N = B->n_sims;
    const int32_t k = t >= 0 ? kk[t] : 0;
    const bool live = t >= 0 && k >= 1 && k <= N;
    // Binomial(35, p) probabilities in float32 from log C(35, y) + y log p + (35 - y) log(1 - p),
    // p = T / 2^32 (the simulated draw rule); p = 0 puts all mass on y = 0
    const float p0 = (float)B->T0[lane >> 3] * 0x1p-32f, p1 = (float)B->T1[lane & 7] * 0x1p-32f;
    const float l0 = logf(p0), m0 = log1pf(-p0), l1 = logf(p1), m1 = log1pf(-p1);
    float lc[B2_N1];   // log y!, then log C(35, y)
    {
        float lfac = 0.0f;
#pragma unroll
        for (int y = 0; y < B2_N1; ++y) {
            if (y > 0) lfac += logf((float)y);
            lc[y] = lfac;
        }
    }
    float b0[B2_N1];
    float run = 0.0f;
    tail1[B2_N1][lane] = 0.0f;
#pragma unroll
    for (int y = B2_N1 - 1; y >= 0; --y) {
        const float c = lc[NP35] - lc[y] - lc[NP35 - y];
        b0[y] = p0 > 0.0f ? expf(c + (float)y * l0 + (float)(NP35 - y) * m0) : (y == 0 ? 1.0f : 0.0f);
        run += p1 > 0.0f ? expf(c + (float)y * l1 + (float)(NP35 - y) * m1) : (y == 0 ? 1.0f : 0.0f);
        tail1[y][lane] = run;
    }
    lds_wave_sync();
    auto below = [&](int g) -> float {   // P(S < S_g) of this lane's tile
        const uint32_t *__restrict__ cw = reinterpret_cast<const uint32_t *>(gcut + (size_t)g * B2_N1);
        uint32_t w[B2_N1 / 4];
#pragma unroll
        for (int i = 0; i < B2_N1 / 4; ++i) w[i] = cw[i];
        float sum = 0.0f;
#pragma unroll
        for (int y0 = 0; y0 < B2_N1; ++y0) sum += b0[y0] * tail1[(w[y0 >> 2] >> (8 * (y0 & 3))) & 0xFFu][lane];
        return sum;
    };
    const float kf = (float)k, sd = sqrtf(kf + 1.0f);
    const float lo_t = kf - zmargin * sd - 2.0f, hi_t = kf + zmargin * sd + 2.0f;
    const float Nf = (float)N;
    int a = 0, b = n_groups;            // lo group: the last g with N P(S < S_g) <= lo_t (g = 0 has 0)
    while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (Nf * below(m) <= lo_t) a = m; else b = m;
    }
    const int glo = a;
    a = -1;
    b = n_groups - 1;                   // hi group: the first g with N P(S <= S_g) >= hi_t
    while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (Nf * below(m + 1) >= hi_t) b = m; else a = m;
    }
    const int ghi = b;
    if (t >= 0) br[t] = make_int2(gstart[glo], gstart[ghi + 1] - 1);
    // cut points of this tile: clo = cut of its first group, chi = cut of the group after its last
    const uint8_t *__restrict__ clo = gcut + (size_t)glo * B2_N1, *__restrict__ chi = gcut + (size_t)(ghi + 1) * B2_N1;
    for (int y0 = 0; y0 < B2_N1; ++y0) {
        cb[lane >> 3][y0][lane & 7] = live ? clo[y0] : (uint8_t)B2_N1;
        cb[lane >> 3][y0][8 + (lane & 7)] = live ? chi[y0] : (uint8_t)B2_N1;
    }
    lds_wave_sync();
    const uint4 *__restrict__ src = reinterpret_cast<const uint4 *>(&cb[0][0][0]);
    uint4 *__restrict__ dst = cut + (size_t)blockIdx.x * B2U * B2_N1;
    for (int i = lane; i < B2U * B2_N1; i += WAVE) dst[i] = src[i];
}

// One workgroup per batch.  Simulations go in rounds of B2_ROUND chunks per wave: the byte-wise
// pass counts the tiles below their bracket and lists the simulations that fall inside some
// tile's bracket (under common random numbers such a simulation is usually inside the brackets
// of many of the batch's neighbouring tiles at once, so a per-lane loop over its tiles would
// stall the wave); after the round the listed simulations are taken one per wave-step with
// lane = tile: position lookup and histogram add without divergence.
constexpr int B2_ROUND = 4;
__global__ __launch_bounds__(SEL_WG) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_b2_select(
    const Blk2 *__restrict__ blocks, const uint4 *__restrict__ recs, const int32_t *__restrict__ kk,
    const int2 *__restrict__ br, const uint4 *__restrict__ cut, const int32_t *__restrict__ S_pos,
    const int32_t *__restrict__ S_order, const int32_t *__restrict__ S_group, const double *__restrict__ S_tbl,
    double *__restrict__ lam, int32_t *__restrict__ rej_at, uint32_t *__restrict__ fb) {
    constexpr int NT = B2U * B2V;
    constexpr int NWV = SEL_WG / WAVE;
    constexpr uint32_t H = 0x80808080u, ONES = 0x01010101u;
    __shared__ uint16_t spos[B2_NOUT];
    __shared__ uint4 ct[B2U][B2_N1];
    __shared__ uint32_t hist[B2_HB];
    __shared__ int2 prm[NT];          // per slot: (first bin - lo, histogram present)
    __shared__ uint32_t below[NT];    // per slot: simulations with S < S(lo)
    __shared__ uint32_t lst[NWV * B2_ROUND * WAVE];   // simulations of the round inside some bracket
    __shared__ uint32_t s_nl;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid >> 6;
    const Blk2 *__restrict__ B = blocks + blockIdx.x;
    const int32_t N = B->n_sims;
    for (int o = tid; o < B2_NOUT; o += SEL_WG) spos[o] = (uint16_t)S_pos[o];
    {
        const uint4 *__restrict__ cs = cut + (size_t)blockIdx.x * B2U * B2_N1;
        for (int i = tid; i < B2U * B2_N1; i += SEL_WG) (&ct[0][0])[i] = cs[i];
    }
    for (int i = tid; i < B2_HB; i += SEL_WG) hist[i] = 0u;
    if (tid == 0) s_nl = 0u;
    // lane = slot for the list pass and the setup: the slot's bracket and histogram region
    int my_lo = 0, my_hi = -1, my_base = 0;
    {
        const int32_t t = B->tile[lane];
        const int32_t k = t >= 0 ? kk[t] : 0;
        int lo = 0, W = 0;
        if (t >= 0 && k >= 1 && k <= N) {
            const int2 b = br[t];
            lo = b.x;
            W = b.y - b.x + 1;
        } else if (t >= 0 && wv == 0) {   // outside Theorem 4's range: +-inf, no selection
            lam[t] = k <= 0 ? -INFINITY : INFINITY;
            rej_at[t] = k <= 0 ? 0 : N;
        }
        int x = W;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            const int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        const int hoff = x - W;
        const bool fits = W > 0 && hoff + W <= B2_HB;   // else: exact full pass
        if (wv == 0) {
            below[lane] = 0u;
            prm[lane] = make_int2(hoff - lo, fits ? 1 : 0);
        }
        if (fits) {
            my_lo = lo;
            my_hi = lo + W - 1;
            my_base = hoff - lo;
        }
    }
    __syncthreads();
    const uint4 *__restrict__ rb = recs + B->key_base;
    const int nch = (N + WAVE - 1) / WAVE;
    uint32_t acc[B2U][2];   // per row and half: packed byte counts of simulations below the bracket
#pragma unroll
    for (int u = 0; u < B2U; ++u) acc[u][0] = acc[u][1] = 0u;
    auto flush = [&]() {    // wave sums of the byte counters (as 16-bit pairs) into below[]
#pragma unroll
        for (int u = 0; u < B2U; ++u)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint32_t ev = acc[u][h] & 0x00FF00FFu, od = (acc[u][h] >> 8) & 0x00FF00FFu;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    ev += __shfl_xor(ev, off);
                    od += __shfl_xor(od, off);
                }
                if (lane == 0) {
                    atomicAdd(&below[u * B2V + 4 * h + 0], ev & 0xFFFFu);
                    atomicAdd(&below[u * B2V + 4 * h + 1], od & 0xFFFFu);
                    atomicAdd(&below[u * B2V + 4 * h + 2], ev >> 16);
                    atomicAdd(&below[u * B2V + 4 * h + 3], od >> 16);
                }
                acc[u][h] = 0u;
            }
    };
    int since = 0;
    // the record of this wave's next chunk is loaded one chunk ahead (records are padded to whole
    // chunks, so a chunk index below nch is always in bounds)
    uint4 rnext = wv < nch ? rb[wv * WAVE + lane] : make_uint4(0u, 0u, 0u, 0u);
    for (int c0 = 0; c0 < nch; c0 += NWV * B2_ROUND) {
        for (int i = 0; i < B2_ROUND; ++i) {
            const int c = c0 + wv + NWV * i;
            if (c >= nch) break;   // uniform over the wave
            const int j = c * WAVE + lane;
            const uint4 r = rnext;
            if (c + NWV < nch) rnext = rb[(c + NWV) * WAVE + lane];
            const uint32_t live = j < N ? ONES : 0u;
            const uint32_t ya = r.z | H, yb = r.w | H;   // y1 of v = 0..3, 4..7, each byte's high bit set
            // byte high bits of ya - clo: y1 >= clo (below the bracket); of ya - chi: y1 >= chi.
            // In the bracket: chi <= y1 < clo, the high bits of the xor of the two differences;
            // the xors are or-ed whole and masked once (their low bits are ignored).
            uint32_t inb = 0u;
#pragma unroll
            for (int u = 0; u < B2U; ++u) {
                const uint32_t y0 = rec_byte(u < 4 ? r.x : r.y, u & 3);
                const uint4 T = ct[u][y0];
                const uint32_t dl = ya - T.x, dh = yb - T.y, el = ya - T.z, eh = yb - T.w;
                acc[u][0] += (dl >> 7) & live;
                acc[u][1] += (dh >> 7) & live;
                inb |= (dl ^ el) | (dh ^ eh);
            }
            const bool in = live != 0u && (inb & H) != 0u;
            const unsigned long long bal = __ballot(in);
            if (bal) {
                uint32_t base = 0u;
                if (lane == 0) base = atomicAdd(&s_nl, (uint32_t)__popcll(bal));
                base = __shfl(base, 0);
                if (in) lst[base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = (uint32_t)j;
            }
            if (++since == 255) {   // byte counters: at most 255 increments between flushes
                flush();
                since = 0;
            }
        }
        __syncthreads();
        // the round's listed simulations, lane = tile: exact position, histogram of the bracket
        const uint32_t nl = s_nl;
        const int u = lane >> 3, v = lane & 7;
        for (uint32_t li = (uint32_t)wv; li < nl; li += NWV) {
            const uint32_t j = __builtin_amdgcn_readfirstlane(lst[li]);
            const uint4 r = rb[j];
            const uint32_t y0 = rec_byte(u < 4 ? r.x : r.y, u & 3), y1 = rec_byte(v < 4 ? r.z : r.w, v & 3);
            const int pos = (int)spos[y0 * B2_N1 + y1];
            if (pos >= my_lo && pos <= my_hi) atomicAdd(&hist[my_base + pos], 1u);
        }
        __syncthreads();
        if (tid == 0) s_nl = 0u;
        __syncthreads();
    }
    flush();
    __syncthreads();
    // per tile: walk the bracket's histogram in position order (one wave per tile)
    for (int s = wv; s < NT; s += SEL_WG / WAVE) {
        const int32_t t = B->tile[s];
        if (t < 0) continue;
        const int32_t k = kk[t];
        if (k <= 0 || k > N) continue;
        const int2 q = prm[s];
        const int2 b = br[t];
        bool done = false;
        const uint32_t bel = below[s];
        if (q.y && bel < (uint32_t)k) {
            const int lo = b.x, W = b.y - b.x + 1, h0 = q.x + lo;
            uint32_t run = bel;
            for (int i0 = 0; i0 < W && !done; i0 += WAVE) {
                const int i = i0 + lane;
                const uint32_t c = i < W ? hist[h0 + i] : 0u;
                uint32_t incl = c;
#pragma unroll
                for (int o = 1; o < WAVE; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o);
                    if (lane >= o) incl += y;
                }
                const uint32_t excl = run + incl - c;
                if (i < W) hist[h0 + i] = excl;   // count strictly before position lo + i
                lds_wave_sync();
                const bool hit = i < W && excl < (uint32_t)k && excl + c >= (uint32_t)k;
                const unsigned long long bal = __ballot(hit);
                if (bal) {
                    if (hit) {
                        const int p = lo + i;
                        const int g = S_group[p];   // >= lo: the bracket starts a tie group
                        lam[t] = S_tbl[S_order[p]];
                        rej_at[t] = (int32_t)hist[h0 + (g - lo)];
                    }
                    done = true;
                }
                run += __shfl(incl, WAVE - 1);
            }
        }
        if (!done && lane == 0) {   // outside the bracket or not histogrammed: exact full pass
            const uint32_t slot = atomicAdd(&fb[0], 1u);
            fb[1 + slot] = (uint32_t)t;
        }
    }
}

// Exact selection from the full histogram of a tile's 1,296 outcomes, for the tiles listed in fb;
// a fixed grid of workgroups takes the listed tiles in turn.
__global__ __launch_bounds__(SEL_WG) void k_b2_full(const uint4 *__restrict__ recs, const int64_t *__restrict__ key_off,
                                                    const int64_t *__restrict__ key_slot,
                                                    const int32_t *__restrict__ N, const int32_t *__restrict__ kk,
                                                    const double *__restrict__ S_tbl,
                                                    const int32_t *__restrict__ S_order,
                                                    const int32_t *__restrict__ S_group,
                                                    const uint32_t *__restrict__ fb, double *__restrict__ lam,
                                                    int32_t *__restrict__ rej_at) {
    __shared__ uint32_t hist[B2_NOUT];
    __shared__ uint32_t cumx[B2_NOUT];   // exclusive cumulative counts in S order
    const int tid = threadIdx.x;
    const uint32_t n_list = fb[0];
    for (uint32_t li = blockIdx.x; li < n_list; li += gridDim.x) {
        const int32_t t = (int32_t)fb[1 + li];
        const int32_t n = N[t], k = kk[t];
        const int s = (int)key_slot[t];
        const uint4 *__restrict__ rb = recs + key_off[t];
        for (int j = tid; j < B2_NOUT; j += SEL_WG) hist[j] = 0u;
        __syncthreads();
        constexpr int LPT = 4;   // records in flight per thread
        for (int j0 = tid; j0 < n; j0 += SEL_WG * LPT) {
            uint4 r[LPT];
#pragma unroll
            for (int l = 0; l < LPT; ++l) {
                const int j = j0 + l * SEL_WG;
                if (j < n) r[l] = rb[j];
            }
#pragma unroll
            for (int l = 0; l < LPT; ++l)
                if (j0 + l * SEL_WG < n) atomicAdd(&hist[rec_outcome(r[l], s)], 1u);
        }
        __syncthreads();
        if (tid < WAVE) {
            uint32_t run = 0u;
            for (int base = 0; base < B2_NOUT; base += WAVE) {
                const int p = base + tid;
                const uint32_t c = p < B2_NOUT ? hist[S_order[p]] : 0u;
                uint32_t incl = c;
#pragma unroll
                for (int o = 1; o < WAVE; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o);
                    if (tid >= o) incl += y;
                }
                const uint32_t excl = run + incl - c;
                if (p < B2_NOUT) cumx[p] = excl;
                lds_wave_sync();
                const bool hit = p < B2_NOUT && excl < (uint32_t)k && excl + c >= (uint32_t)k;
                if (__ballot(hit)) {
                    if (hit) {
                        lam[t] = S_tbl[S_order[p]];
                        rej_at[t] = (int32_t)cumx[S_group[p]];
                    }
                    break;
                }
                run += __shfl(incl, WAVE - 1);
            }
        }
        __syncthreads();   // hist and cumx are rewritten for the next listed tile
    }
}

// ---- continuous statistic (float32 keys): three-pass radix selection (11/11/10 bits) ----
__device__ __forceinline__ uint32_t f2ord(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// k-th smallest (k >= 1) of the n order-preserving keys get(j), j < n, by three radix passes
// (11/11/10 bits) with an LDS histogram; also the number of keys strictly below it.  With
// PASSES = 2 only the top 22 bits are resolved: key is then the smallest value of the 1024-wide
// bin that holds the k-th smallest, and below counts the keys under that bin.  Called by the
// whole workgroup.
template <int PASSES = 3, class Get>
__device__ void radix_kth(int n, uint32_t k, Get get, uint32_t *hist, uint32_t *part, uint32_t *s_bin,
                          uint32_t *s_below, uint32_t &key, uint32_t &below_out) {
    constexpr int BINS = 2048;
    const int tid = threadIdx.x;
    uint32_t prefix = 0u, below = 0u, need = k;
    const int shifts[3] = {21, 10, 0};
    const int widths[3] = {11, 11, 10};
    for (int pass = 0; pass < PASSES; ++pass) {
        const int sh = shifts[pass], wd = widths[pass];
        const uint32_t mask_hi = pass == 0 ? 0u : (0xFFFFFFFFu << (sh + wd));
        for (int j = tid; j < BINS; j += SEL_WG) hist[j] = 0u;
        __syncthreads();
        for (int j = tid; j < n; j += SEL_WG) {
            const uint32_t u = get(j);
            if ((u & mask_hi) == prefix) atomicAdd(&hist[(u >> sh) & ((1u << wd) - 1u)], 1u);
        }
        __syncthreads();
        const int nb = 1 << wd;
        const int per = nb / SEL_WG;
        uint32_t local = 0u;
        for (int j = tid * per; j < (tid + 1) * per; ++j) local += hist[j];
        block_exclusive_scan(local, part);
        uint32_t run = part[tid];
        for (int j = tid * per; j < (tid + 1) * per; ++j) {
            if (run < need && run + hist[j] >= need) {
                *s_bin = (uint32_t)j;
                *s_below = run;
            }
            run += hist[j];
        }
        __syncthreads();
        prefix |= *s_bin << sh;
        below += *s_below;
        need -= *s_below;
        __syncthreads();
    }
    key = prefix;
    below_out = below;
}

// Selection of lambda*_i for float32 keys.  Tiles of at most SEL_SAMPLE keys are selected in
// LDS.  Larger tiles: the first SEL_SAMPLE simulations (i.i.d. draws of the statistic) give
// sample order statistics lo, hi that bracket rank k/N with a margin of z binomial standard
// deviations (z = 5, lowered to no less than 3 where the expected number of keys in the
// bracket would exceed SEL_FILL of the SEL_CAND candidate slots); one pass over the tile's
// keys counts those below lo and keeps those in [lo, hi] in per-thread LDS slots, compacted
// afterwards; if the k-th smallest lies among them it is selected there, else (bracket missed,
// a thread's slots or the candidate buffer full) the exact radix passes run over HBM.  Either
// way the result is the exact k-th smallest key.
constexpr int SEL_SAMPLE = 2048;
constexpr int SEL_CAND = 2048;
// candidate slots per thread in the pass over the tile (the last one takes the keys outside the
// bracket), and the share of SEL_CAND the bracket aims to fill: at 0.45 a thread of a
// 32,768-key tile expects 3.6 bracket keys, and more than 15 has probability ~1e-7
constexpr int SEL_TSLOTS = 16;
constexpr double SEL_FILL = 0.45;

template <bool VEC4>
__global__ __launch_bounds__(SEL_WG) void k_select_f32(const float *__restrict__ keys,
                                                       const int64_t *__restrict__ key_off,
                                                       const int64_t *__restrict__ key_stride,
                                                       const int32_t *__restrict__ N,
                                                       const int32_t *__restrict__ kk,
                                                       double *__restrict__ lam,
                                                       int32_t *__restrict__ rej_at) {
    // hist (radix passes) and the per-thread candidate slots of the pass over the tile share
    // one buffer: the pass runs between the bracket's radix passes and the final one
    __shared__ uint32_t hist_slots[SEL_TSLOTS * SEL_WG > 2048 ? SEL_TSLOTS * SEL_WG : 2048];
    uint32_t *const hist = hist_slots, *const slots = hist_slots;
    __shared__ uint32_t part[SEL_WG];
    // the sample is used up (bracket chosen) before the pass fills the candidates: one buffer
    __shared__ uint32_t samp_cand[SEL_CAND > SEL_SAMPLE ? SEL_CAND : SEL_SAMPLE];
    uint32_t *const samp = samp_cand, *const cand = samp_cand;
    __shared__ uint32_t s_bin, s_below, s_lt, s_over;
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int32_t n = N[t];
    const int32_t k = kk[t];
    if (k <= 0 || k > n) {
        if (tid == 0) {
            lam[t] = k <= 0 ? -INFINITY : INFINITY;
            if (rej_at) rej_at[t] = k <= 0 ? 0 : n;
        }
        return;
    }
    // key of simulation j at kt + (j / 64) * stride + j % 64 (chunked layouts; stride 64 = contiguous)
    const float *__restrict__ kt = keys + key_off[t];
    const int64_t stride = key_stride[t];
    auto hbm = [&](int j) { return f2ord(kt[(int64_t)(j >> 6) * stride + (j & 63)]); };
    auto from_samp = [&](int j) { return samp[j]; };
    auto from_cand = [&](int j) { return cand[j]; };
    const int m = n < SEL_SAMPLE ? n : SEL_SAMPLE;
#pragma unroll
    for (int i = 0; i < SEL_SAMPLE / SEL_WG; ++i) {
        const int j = i * SEL_WG + tid;
        if (j < m) samp[j] = hbm(j);
    }
    __syncthreads();
    uint32_t key = 0u, below = 0u;
    if (n <= SEL_SAMPLE) {
        radix_kth(n, (uint32_t)k, from_samp, hist, part, &s_bin, &s_below, key, below);
    } else {
        const double pr = (double)k / (double)n;
        const double sd = sqrt((double)m * pr * (1.0 - pr));
        // expected keys in the bracket: n (2 z sd + 2) / m
        const double z_fit = (SEL_FILL * SEL_CAND * m / (double)n - 2.0) / (2.0 * sd);
        const double z = fmin(5.0, fmax(3.0, z_fit));
        const int lo_r = (int)floor(pr * m - z * sd) - 1;   // sample ranks (1-based) of the bracket
        const int hi_r = (int)ceil(pr * m + z * sd) + 1;
        // the bracket is widened to the 22-bit bins that hold those sample order statistics
        // (two radix passes each instead of three; a few more candidates, the same result)
        uint32_t lo = 0u, hi = 0xFFFFFFFFu, dummy = 0u;
        if (lo_r >= 1) radix_kth<2>(m, (uint32_t)lo_r, from_samp, hist, part, &s_bin, &s_below, lo, dummy);
        if (hi_r <= m) {
            radix_kth<2>(m, (uint32_t)hi_r, from_samp, hist, part, &s_bin, &s_below, hi, dummy);
            hi |= 0x3FFu;
        }
        if (tid == 0) {
            s_lt = 0u;
            s_over = 0u;
        }
        __syncthreads();
        // one pass over the tile: count below the bracket, keep the bracket's keys.  Each
        // thread loads a batch of keys before using any (many loads in flight; with VEC4 the
        // tile's 64-key chunks are 256-byte aligned and read as float4).  Every key is written,
        // without a branch, to the thread's next free slot when it lies in the bracket and to
        // the thread's last slot (scratch) otherwise; a thread with more than SEL_TSLOTS - 1
        // bracket keys sends the tile to the exact path.
        // lt: this wave's keys below the bracket (the same in every lane); per key two compares,
        // scalar adds for the count, and the slot store
        // nin_w: this wave's keys in the bracket; a thread whose bracket keys outnumber its
        // SEL_TSLOTS - 1 slots makes the wave's filled slots fall short of nin_w
        uint32_t lt = 0u, nin_w = 0u;
        char *const sbase = reinterpret_cast<char *>(slots);
        const uint32_t scratch_off = (uint32_t)(((SEL_TSLOTS - 1) * SEL_WG + tid) * 4);
        uint32_t next_off = (uint32_t)(tid * 4);   // byte offset of the thread's next free slot (stops at the scratch slot)
        auto take = [&](uint32_t u, bool valid) {
            const bool ge = u >= lo, le = u <= hi;
            const bool in = valid && ge && le;
            lt += (uint32_t)__popcll(__ballot(valid && !ge));
            nin_w += (uint32_t)__popcll(__ballot(in));
            *reinterpret_cast<uint32_t *>(sbase + (in ? next_off : scratch_off)) = u;
            next_off = min(next_off + (in ? (uint32_t)(SEL_WG * 4) : 0u), scratch_off);
        };
        if (VEC4) {
            // the 4-arm and basket keys are 1 - P >= +0 (min over arms of float64 values in
            // [0, 1], rounded): their order key is the bit pattern with the sign bit set, which
            // is f2ord for non-negative floats (the sample and the exact paths keep f2ord)
            auto ord_nn = [](float x) { return __float_as_uint(x) ^ 0x80000000u; };
            constexpr int QB = 4;   // float4 per thread per round: 16 keys
            const int nq = ((n + 63) >> 6) * 16;
            for (int q0 = 0; q0 < nq; q0 += SEL_WG * QB) {
                float4 v[QB];
#pragma unroll
                for (int i = 0; i < QB; ++i) {
                    const int q = q0 + i * SEL_WG + tid;
                    v[i] = q < nq ? *reinterpret_cast<const float4 *>(kt + (int64_t)(q >> 4) * stride + (q & 15) * 4)
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
                }
                if (4 * (q0 + SEL_WG * QB) <= n) {   // uniform: every key of the round is a simulation's
#pragma unroll
                    for (int i = 0; i < QB; ++i) {
                        take(ord_nn(v[i].x), true);
                        take(ord_nn(v[i].y), true);
                        take(ord_nn(v[i].z), true);
                        take(ord_nn(v[i].w), true);
                    }
                    continue;
                }
#pragma unroll
                for (int i = 0; i < QB; ++i) {
                    const int j = 4 * (q0 + i * SEL_WG + tid);
                    take(ord_nn(v[i].x), j + 0 < n);
                    take(ord_nn(v[i].y), j + 1 < n);
                    take(ord_nn(v[i].z), j + 2 < n);
                    take(ord_nn(v[i].w), j + 3 < n);
                }
            }
        } else {
            constexpr int SEL_BATCH = 8;
            for (int j0 = 0; j0 < n; j0 += SEL_WG * SEL_BATCH) {
                uint32_t u[SEL_BATCH];
#pragma unroll
                for (int i = 0; i < SEL_BATCH; ++i) {
                    const int j = j0 + i * SEL_WG + tid;
                    u[i] = j < n ? hbm(j) : 0u;
                }
#pragma unroll
                for (int i = 0; i < SEL_BATCH; ++i) take(u[i], j0 + i * SEL_WG + tid < n);
            }
        }
        // the threads' bracket keys, compacted into the candidate buffer in thread order
        const uint32_t mine = (next_off - (uint32_t)(tid * 4)) / (uint32_t)(SEL_WG * 4);
        uint32_t filled = mine;
        for (int off = 32; off >= 1; off >>= 1) filled += __shfl_xor(filled, off);
        if (lane == 0) {
            atomicAdd(&s_lt, lt);
            if (filled != nin_w) s_over = 1u;   // some thread ran out of slots
        }
        block_exclusive_scan(mine, part);   // synchronises: s_lt and s_over are complete after it
        const uint32_t off = part[tid];
        if (tid == SEL_WG - 1) s_bin = off + mine;   // total, through a spare word
        __syncthreads();
        const uint32_t nc = s_over ? 0xFFFFFFFFu : s_bin, nlt = s_lt;
        if (nc <= (uint32_t)SEL_CAND)
            for (uint32_t j = 0; j < mine; ++j) cand[off + j] = slots[j * SEL_WG + tid];
        __syncthreads();
        if (nc <= (uint32_t)SEL_CAND && nlt < (uint32_t)k && (uint32_t)k <= nlt + nc) {
            radix_kth((int)nc, (uint32_t)k - nlt, from_cand, hist, part, &s_bin, &s_below, key, below);
            below += nlt;
        } else {
            radix_kth(n, (uint32_t)k, hbm, hist, part, &s_bin, &s_below, key, below);   // exact fallback
        }
    }
    if (tid == 0) {
        lam[t] = (double)ord2f(key);
        if (rej_at) rej_at[t] = (int32_t)below;
    }
}

// ---- 4-arm design, bracketed keys ----
// The pilot pass stores the float32 keys of the first H4_PILOT simulations.  k_h4_bracket takes
// them as the sample of k_select_f32 (order statistics of rank (k/N) m -+ z sd, widened to 22-bit
// bins, z at most the margin and lowered towards 3 so that the bracket expects at most H4_FILL of
// the H4_SELCAND candidate slots), counts the pilot keys below the bracket and keeps those in it;
// tiles of at most H4_PILOT simulations are selected there and then.  The fused pass over the
// other simulations adds its own counts and candidates (k_hier4, KEYS = 2).  k_h4_select then
// finds the k-th smallest key among the candidates when it lies there (count below < k <= count
// below + candidates, no region overflowed); otherwise it takes three radix passes over the tile's
// keys regenerated one by one from the counter-based generator (the fused pass's arithmetic on
// the tile's own thresholds), so the result is the exact k-th smallest key either way.
constexpr int H4_SELCAND = 4096;
constexpr double H4_FILL = 0.45;

__global__ __launch_bounds__(SEL_WG) void k_h4_bracket(const float *__restrict__ keys,
                                                       const int64_t *__restrict__ key_off,
                                                       const int64_t *__restrict__ key_stride,
                                                       const int32_t *__restrict__ N, const int32_t *__restrict__ kk,
                                                       float margin, int32_t maxs, int64_t tot,
                                                       float2 *__restrict__ brk, uint32_t *__restrict__ below,
                                                       uint32_t *__restrict__ cnt, float *__restrict__ cand,
                                                       double *__restrict__ lam, int32_t *__restrict__ rej_at) {
    __shared__ uint32_t hist[2048];
    __shared__ uint32_t part[SEL_WG];
    __shared__ uint32_t samp[H4_PILOT];
    __shared__ uint32_t s_bin, s_below, s_lt, s_in;
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x;
    const int32_t n = N[t];
    const int32_t k = kk[t];
    uint32_t *__restrict__ ct = cnt + t * (int64_t)(maxs + 1);
    for (int i = tid; i <= maxs; i += SEL_WG) ct[i] = 0u;   // the pass's regions start empty
    const float2 none = make_float2(-INFINITY, -INFINITY);    // no key below or inside
    if (k <= 0 || k > n) {   // outside Theorem 4's range: -+inf, no selection
        if (tid == 0) {
            lam[t] = k <= 0 ? -INFINITY : INFINITY;
            if (rej_at) rej_at[t] = k <= 0 ? 0 : n;
            brk[t] = none;
            below[t] = 0u;
        }
        return;
    }
    const float *__restrict__ kt = keys + key_off[t];
    const int64_t stride = key_stride[t];
    const int m = n < H4_PILOT ? n : H4_PILOT;
    for (int j = tid; j < m; j += SEL_WG) samp[j] = f2ord(kt[(int64_t)(j >> 6) * stride + (j & 63)]);
    __syncthreads();
    auto from_samp = [&](int j) { return samp[j]; };
    if (n <= H4_PILOT) {   // the pilot is the whole tile
        uint32_t key = 0u, bel = 0u;
        radix_kth(n, (uint32_t)k, from_samp, hist, part, &s_bin, &s_below, key, bel);
        if (tid == 0) {
            lam[t] = (double)ord2f(key);
            if (rej_at) rej_at[t] = (int32_t)bel;
            brk[t] = none;
            below[t] = 0u;
        }
        return;
    }
    const double pr = (double)k / (double)n;
    const double sd = sqrt((double)m * pr * (1.0 - pr));
    const double z_fit = (H4_FILL * H4_SELCAND * m / (double)n - 2.0) / (2.0 * sd);
    const double z = fmin((double)margin, fmax(3.0, z_fit));
    const int lo_r = (int)floor(pr * m - z * sd) - 1;
    const int hi_r = (int)ceil(pr * m + z * sd) + 1;
    uint32_t lo = 0u, hi = 0xFFFFFFFFu, dummy = 0u;
    if (lo_r >= 1) radix_kth<2>(m, (uint32_t)lo_r, from_samp, hist, part, &s_bin, &s_below, lo, dummy);
    if (hi_r <= m) {
        radix_kth<2>(m, (uint32_t)hi_r, from_samp, hist, part, &s_bin, &s_below, hi, dummy);
        hi |= 0x3FFu;
    }
    // float bounds, compared as the fused pass compares them
    const float lo_f = lo_r >= 1 ? ord2f(lo) : -INFINITY;
    const float hi_f = hi_r <= m ? ord2f(hi) : INFINITY;
    if (tid == 0) {
        s_lt = 0u;
        s_in = 0u;
    }
    __syncthreads();
    uint32_t lt = 0u;
    float *__restrict__ cp = cand + t * tot;   // the pilot's region
    for (int j = tid; j < m; j += SEL_WG) {
        const float v = ord2f(samp[j]);
        if (v < lo_f) {
            ++lt;
        } else if (v <= hi_f) {
            const uint32_t p = atomicAdd(&s_in, 1u);
            if (p < (uint32_t)H4_PCAP) cp[p] = v;
        }
    }
    if (lt) atomicAdd(&s_lt, lt);
    __syncthreads();
    if (tid == 0) {
        below[t] = s_lt;
        ct[0] = s_in;   // more than H4_PCAP: the tile takes the exact path
        brk[t] = make_float2(lo_f, hi_f);
    }
}

// The 4-arm statistic of simulation k at one tile (thresholds T of the four arms, configuration
// b): the fused pass's arithmetic for that single (simulation, tile).
__device__ __forceinline__ float h4_regen_key(uint32_t k, const uint32_t T[4], uint32_t b, uint32_t key0,
                                              uint32_t key1, const float4 *__restrict__ tbl) {
    constexpr int M1 = NP35 + 1;
    int y[4] = {0, 0, 0, 0};
#pragma unroll
    for (int blk = 0; blk < NP35; ++blk) {   // 4 arms x 35 words = 35 blocks; word w is arm w / 35's
        const u32x4 w = philox_block((uint32_t)blk, k, key0, key1);
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int a = (4 * blk + l) / NP35;
            y[a] += (u32x4_get(w, l) < T[a]) ? 1 : 0;
        }
    }
    const float4 q = tbl[((y[0] * M1 + y[1]) * M1 + y[2]) * M1 + y[3]];
    float sb = INFINITY;
    if (b & 1u) sb = fminf(sb, q.x);
    if (b & 2u) sb = fminf(sb, q.y);
    if (b & 4u) sb = fminf(sb, q.z);
    return sb;
}

__global__ __launch_bounds__(SEL_WG) void k_h4_select(const int32_t *__restrict__ N, const int32_t *__restrict__ kk,
                                                      const uint32_t *__restrict__ below,
                                                      const uint32_t *__restrict__ cnt, const float *__restrict__ cand,
                                                      int32_t maxs, int32_t caps, int64_t tot,
                                                      const uint32_t *__restrict__ tileT,
                                                      const int32_t *__restrict__ cfg,
                                                      const float4 *__restrict__ tbl, uint32_t key0, uint32_t key1,
                                                      uint32_t *__restrict__ fb, double *__restrict__ lam,
                                                      int32_t *__restrict__ rej_at) {
    __shared__ uint32_t hist[2048];
    __shared__ uint32_t part[SEL_WG];
    __shared__ uint32_t cbuf[H4_SELCAND];
    __shared__ uint32_t spre[H4_MAXS + 2];   // first candidate of each region in cbuf
    __shared__ uint32_t s_bin, s_below, s_over;
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x;
    const int32_t n = N[t];
    const int32_t k = kk[t];
    if (k <= 0 || k > n || n <= H4_PILOT) return;   // selected by k_h4_bracket
    const uint32_t *__restrict__ ct = cnt + t * (int64_t)(maxs + 1);
    if (tid == 0) s_over = 0u;
    __syncthreads();
    uint32_t run = 0u;   // the same in every thread
    for (int base = 0; base <= maxs; base += SEL_WG) {
        const int r = base + tid;
        const uint32_t c = r <= maxs ? ct[r] : 0u;
        if (r <= maxs && c > (r == 0 ? (uint32_t)H4_PCAP : (uint32_t)caps)) s_over = 1u;   // some keys were not kept
        block_exclusive_scan(c, part);
        if (r <= maxs) spre[r] = run + part[tid];
        if (tid == SEL_WG - 1) s_bin = part[tid] + c;
        __syncthreads();
        run += s_bin;
        __syncthreads();
    }
    if (tid == 0) spre[maxs + 1] = run;
    const uint32_t bl = below[t];
    __syncthreads();
    uint32_t key = 0u, bel = 0u;
    if (!s_over && run <= (uint32_t)H4_SELCAND && bl < (uint32_t)k && (uint32_t)k <= bl + run) {
        const float *__restrict__ cp = cand + t * tot;
        for (uint32_t i = tid; i < run; i += SEL_WG) {
            int a = 0, b = maxs + 1;   // region: spre[a] <= i < spre[a + 1]
            while (b - a > 1) {
                const int mid = (a + b) >> 1;
                if (spre[mid] <= i)
                    a = mid;
                else
                    b = mid;
            }
            const uint32_t j = i - spre[a];
            const int64_t off = a == 0 ? (int64_t)j : (int64_t)H4_PCAP + (int64_t)(a - 1) * caps + j;
            cbuf[i] = f2ord(cp[off]);
        }
        __syncthreads();
        radix_kth((int)run, (uint32_t)k - bl, [&](int j) { return cbuf[j]; }, hist, part, &s_bin, &s_below, key, bel);
        bel += bl;
    } else {
        if (tid == 0) fb[1 + atomicAdd(&fb[0], 1u)] = (uint32_t)t;
        uint32_t T[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) T[a] = tileT[4 * t + a];
        const uint32_t b = (uint32_t)cfg[t];
        radix_kth(n, (uint32_t)k, [&](int j) { return f2ord(h4_regen_key((uint32_t)j, T, b, key0, key1, tbl)); },
                  hist, part, &s_bin, &s_below, key, bel);
    }
    if (tid == 0) {
        lam[t] = (double)ord2f(key);
        if (rej_at) rej_at[t] = (int32_t)bel;
    }
}

// ---- randomised calibration: the statistic is the pair (S, u), u the simulation's adjoined
// uniform (philox_tiebreak), ordered lexicographically.  Given the k-th smallest S, lambda, and
// the count `below` of keys strictly under it (the selection's outputs), the k-th smallest pair
// is (lambda, c) with c the (k - below)-th smallest u among the simulations whose key equals
// lambda.  The tied simulations' u are regenerated from the counter and gathered in LDS; more
// than TB_CAND ties fall back to radix passes over the whole tile with every non-tied key
// mapped to 0xFFFFFFFF (which cannot change a rank <= the number of ties).  On exit rej_at[t]
// holds the number of pairs strictly below (lambda, c).
// Key layouts: TB_F32 float32 keys at kt[(j / 64) * stride + j % 64]; TB_F32V4 the same with
// 256-byte aligned 64-key chunks (read as float4).  The 2-arm designs' records serve a batch of
// tiles at once and take the batch-level kernel below instead.
enum { TB_F32 = 0, TB_F32V4 = 1 };
constexpr int TB_RANK = 512;          // tie classes up to this size are ranked by counting
constexpr int TB_CAND = 4096;         // tied simulations gathered in LDS

template <int MODE>
__global__ __launch_bounds__(SEL_WG) void k_tiebreak(const void *__restrict__ keys_,
                                                     const int64_t *__restrict__ key_off,
                                                     const int64_t *__restrict__ key_stride,
                                                     const int32_t *__restrict__ N,
                                                     const int32_t *__restrict__ kk,
                                                     const double *__restrict__ lam, uint32_t key0,
                                                     uint32_t key1, int32_t *__restrict__ rej_at,
                                                     uint32_t *__restrict__ c_out) {
    __shared__ uint32_t hist[2048];
    __shared__ uint32_t part[SEL_WG];
    __shared__ uint32_t cand[TB_CAND];
    __shared__ uint32_t s_bin, s_below, s_cnt;
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int32_t n = N[t];
    const int32_t k = kk[t];
    if (k <= 0 || k > n) {
        if (tid == 0) c_out[t] = k <= 0 ? 0u : 0xFFFFFFFFu;
        return;
    }
    const double L = lam[t];
    const uint32_t Lord = f2ord((float)L);
    const uint32_t below_lam = (uint32_t)rej_at[t];
    const uint32_t need = (uint32_t)k - below_lam;   // >= 1: the k-th key is a tie
    const int64_t stride = key_stride[t];
    const float *__restrict__ kf = (const float *)keys_ + key_off[t];
    if (tid == 0) s_cnt = 0u;
    __syncthreads();
    auto tied = [&](int j) -> bool { return f2ord(kf[(int64_t)(j >> 6) * stride + (j & 63)]) == Lord; };
    // append simulation j's uniform when `in` (called by every lane of the wave)
    auto take = [&](bool in, int j) {
        const unsigned long long bal = __ballot(in);
        if (bal) {   // uniform
            uint32_t base = 0u;
            if (lane == 0) base = atomicAdd(&s_cnt, (uint32_t)__popcll(bal));
            base = __shfl(base, 0);
            const uint32_t pos = base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
            if (in && pos < (uint32_t)TB_CAND) cand[pos] = philox_tiebreak((uint32_t)j, key0, key1);
        }
    };
    // one pass over the tile with several 16-byte (or 4-byte) loads in flight per thread; trip
    // counts are uniform so that every lane takes part in the ballots
    constexpr int LB = 4;
    if (MODE == TB_F32V4) {
        const int nq = ((n + 63) >> 6) * 16;   // float4 pieces
        for (int q0 = 0; q0 < nq; q0 += SEL_WG * LB) {
            float4 v[LB];
#pragma unroll
            for (int i = 0; i < LB; ++i) {
                const int q = q0 + i * SEL_WG + tid;
                v[i] = q < nq ? *reinterpret_cast<const float4 *>(kf + (int64_t)(q >> 4) * stride + (q & 15) * 4)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int i = 0; i < LB; ++i) {
                const int q = q0 + i * SEL_WG + tid;
                const int j0 = 4 * q;
                const bool ok = q < nq;
                take(ok && j0 + 0 < n && f2ord(v[i].x) == Lord, j0 + 0);
                take(ok && j0 + 1 < n && f2ord(v[i].y) == Lord, j0 + 1);
                take(ok && j0 + 2 < n && f2ord(v[i].z) == Lord, j0 + 2);
                take(ok && j0 + 3 < n && f2ord(v[i].w) == Lord, j0 + 3);
            }
        }
    } else {
        constexpr int LS = 8;
        for (int j0 = 0; j0 < n; j0 += SEL_WG * LS) {
            uint32_t u[LS];
#pragma unroll
            for (int i = 0; i < LS; ++i) {
                const int j = j0 + i * SEL_WG + tid;
                u[i] = j < n ? f2ord(kf[(int64_t)(j >> 6) * stride + (j & 63)]) : 0u;
            }
#pragma unroll
            for (int i = 0; i < LS; ++i) {
                const int j = j0 + i * SEL_WG + tid;
                take(j < n && u[i] == Lord, j);
            }
        }
    }
    __syncthreads();
    const uint32_t m = s_cnt;
    uint32_t c = 0u, below_u = 0u;
    if (m <= (uint32_t)TB_RANK) {
        // few ties: the candidate whose rank (smaller values, then equal values at lower
        // positions) is need - 1 is the answer; one pass, no histograms
        for (uint32_t i = (uint32_t)tid; i < m; i += SEL_WG) {
            const uint32_t x = cand[i];
            uint32_t lt = 0u, eq_before = 0u;
            for (uint32_t j = 0; j < m; ++j) {
                const uint32_t y = cand[j];
                lt += y < x ? 1u : 0u;
                eq_before += (y == x && j < i) ? 1u : 0u;
            }
            if (lt + eq_before == need - 1u) {
                s_bin = x;
                s_below = lt;
            }
        }
        __syncthreads();
        c = s_bin;
        below_u = s_below;
    } else if (m <= (uint32_t)TB_CAND) {
        auto from_cand = [&](int j) { return cand[j]; };
        radix_kth((int)m, need, from_cand, hist, part, &s_bin, &s_below, c, below_u);
    } else {
        // more ties than LDS holds: radix passes over the whole tile, non-tied keys mapped to
        // 0xFFFFFFFF (cannot change a rank <= the number of ties)
        auto all = [&](int j) { return tied(j) ? philox_tiebreak((uint32_t)j, key0, key1) : 0xFFFFFFFFu; };
        radix_kth(n, need, all, hist, part, &s_bin, &s_below, c, below_u);
    }
    if (tid == 0) {
        c_out[t] = c;
        rej_at[t] = (int32_t)(below_lam + below_u);
    }
}

// 2-arm designs: the tie-break of a whole batch in one workgroup, each record read once per pass.
// Tile (u, v)'s simulation is tied at lambda iff its outcome lies in lambda's tie group g; as S
// does not increase with y1 for fixed y0, that is cut_{g+1}(y0) <= y1 < cut_g(y0) (the tie-group
// cut table), so one LDS read per row and simulation classifies the row's 8 tiles by byte-wise
// compares, as in the plain selection.  k_b2_tiecut finds each tile's group (one wave per batch,
// lane = slot) and writes the batch's tie ranges over the selection's cut bytes, which are free
// once lambda is known.  A tied simulation's uniform then goes to the tiles it ties:
//  * first pass: into a fixed LDS region of TBB_CAPT words per tile, with an exact count; tiles
//    with at most TBB_CAPT ties pick c by counting ranks there;
//  * the other tiles continue with 8-bit radix passes over their tied uniforms (per-tile
//    histograms), and once every remaining tile's candidate bin is small, one pass gathers the
//    bins' uniforms into LDS and ranks them.
// The result is the exact (need)-th smallest uniform among the tied simulations either way.
constexpr int TBB_WG = 512;
constexpr int TBB_CAPT = 256;                  // uniforms per tile in the first pass
constexpr int TBB_BUF = B2U * B2V * TBB_CAPT;  // 16,384 words: first-pass regions, histograms, gathers
constexpr int TBB_RANK = 512;                  // largest candidate bin ranked by counting
constexpr int TBB_DEPTH = 4;                   // record loads in flight per lane

__global__ __launch_bounds__(WAVE) void k_b2_tiecut(const Blk2 *__restrict__ blocks, const int32_t *__restrict__ kk,
                                                    const double *__restrict__ lam, const double *__restrict__ S_tbl,
                                                    const int32_t *__restrict__ S_order,
                                                    const int32_t *__restrict__ gstart,
                                                    const uint8_t *__restrict__ gcut, int n_groups,
                                                    uint4 *__restrict__ cut, uint32_t *__restrict__ c_out) {
    __shared__ uint8_t cb[B2U][B2_N1][16];   // per row and y0: lo of the 8 tiles, then hi
    const int lane = threadIdx.x;
    const Blk2 *__restrict__ B = blocks + blockIdx.x;
    const int32_t t = B->tile[lane];
    const int32_t N = B->n_sims;
    bool live = false;
    int g = 0;
    if (t >= 0) {
        const int32_t k = kk[t];
        if (k <= 0 || k > N) {
            c_out[t] = k <= 0 ? 0u : 0xFFFFFFFFu;
        } else {
            const double L = lam[t];
            int a = 0, b = n_groups - 1;   // the group whose value is lambda (groups ascend)
            while (a < b) {
                const int m = (a + b) >> 1;
                if (S_tbl[S_order[gstart[m]]] < L) a = m + 1; else b = m;
            }
            g = a;
            live = S_tbl[S_order[gstart[g]]] == L;   // else no tie class: the tie-break writes c = max
        }
    }
    const int u = lane >> 3, v = lane & 7;
    for (int y0 = 0; y0 < B2_N1; ++y0) {   // empty ranges (lo = hi = 0) for slots without ties
        cb[u][y0][v] = live ? gcut[(size_t)(g + 1) * B2_N1 + y0] : (uint8_t)0;
        cb[u][y0][8 + v] = live ? gcut[(size_t)g * B2_N1 + y0] : (uint8_t)0;
    }
    lds_wave_sync();
    const uint4 *__restrict__ src = reinterpret_cast<const uint4 *>(&cb[0][0][0]);
    uint4 *__restrict__ dst = cut + (size_t)blockIdx.x * B2U * B2_N1;
    for (int i = lane; i < B2U * B2_N1; i += WAVE) dst[i] = src[i];
}

// Per wave, tied simulations are first listed in LDS (index and 64-bit slot mask) and taken 64
// at a time, one per lane, so that the uniform is drawn and the slots are visited only for
// simulations tied somewhere (most simulations of a chunk are tied nowhere).
struct TbbList {
    uint32_t j[TBB_WG / WAVE][WAVE];
    uint64_t m[TBB_WG / WAVE][WAVE];
};

template <int MODE>   // 0 first pass, 1 histogram of the next 8 bits, 2 gather
__device__ __forceinline__ void tbb_take(uint32_t j, uint64_t m, uint32_t *buf, uint32_t *fill, const uint32_t *pre,
                                         const uint32_t *off, const uint32_t *cnt, int lvl, uint32_t key0,
                                         uint32_t key1) {
    const uint32_t x = philox_tiebreak(j, key0, key1);
    while (m) {
        const int b = __builtin_ctzll(m);   // bit 8 v + u of slot (u, v)
        m &= m - 1ull;
        const int s = ((b & 7) << 3) | (b >> 3);
        if (MODE == 0) {
            const uint32_t p = atomicAdd(&fill[s], 1u);
            if (p < (uint32_t)TBB_CAPT) buf[s * TBB_CAPT + p] = x;
        } else if ((uint32_t)((uint64_t)x >> (32 - lvl)) == pre[s]) {
            if (MODE == 1) {
                atomicAdd(&buf[s * 256 + ((x >> (24 - lvl)) & 255u)], 1u);
            } else {
                const uint32_t p = atomicAdd(&fill[s], 1u);
                if (p < cnt[s]) buf[off[s] + p] = x;   // cnt[s] of them by construction
            }
        }
    }
}

template <int MODE>
__device__ __forceinline__ void tbb_sweep(const uint4 *__restrict__ rb, int N, const uint4 (*ct)[B2_N1],
                                          TbbList &L, uint32_t *buf, uint32_t *fill, const uint32_t *pre,
                                          const uint32_t *off, const uint32_t *cnt, int lvl, uint32_t key0,
                                          uint32_t key1) {
    constexpr int NWV = TBB_WG / WAVE;
    constexpr uint32_t H = 0x80808080u;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x >> 6;
    const int nch = (N + WAVE - 1) / WAVE;
    int nl = 0;   // listed simulations of this wave (uniform)
    for (int c0 = wv; c0 < nch; c0 += NWV * TBB_DEPTH) {
        uint4 r[TBB_DEPTH];
#pragma unroll
        for (int i = 0; i < TBB_DEPTH; ++i) {   // records padded to whole chunks
            const int c = c0 + NWV * i;
            r[i] = c < nch ? rb[c * WAVE + lane] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int i = 0; i < TBB_DEPTH; ++i) {
            const int c = c0 + NWV * i;
            if (c >= nch) break;   // uniform over the wave
            const int j = c * WAVE + lane;
            const uint32_t ya = r[i].z | H, yb = r[i].w | H;
            // tied: y1 >= lo and not y1 >= hi, byte-wise; row u's flags (bits 7, 15, 23, 31 for
            // v = 0..3 or 4..7) shifted to bits u, 8 + u, ...: bit 8 v + u of the slot mask
            uint32_t ma = 0u, mb = 0u;
#pragma unroll
            for (int u = 0; u < B2U; ++u) {
                const uint32_t y0 = rec_byte(u < 4 ? r[i].x : r[i].y, u & 3);
                const uint4 T = ct[u][y0];
                ma |= ((ya - T.x) & ~(ya - T.z) & H) >> (7 - u);
                mb |= ((yb - T.y) & ~(yb - T.w) & H) >> (7 - u);
            }
            const bool tied = j < N && (ma | mb) != 0u;
            const unsigned long long bal = __ballot(tied);
            if (bal == 0ull) continue;   // uniform
            const int n = __popcll(bal);
            const int rk = (int)__popcll(bal & ((1ull << lane) - 1ull));
            const int first = min(n, WAVE - nl);
            const uint64_t m = (uint64_t)ma | ((uint64_t)mb << 32);
            if (tied && rk < first) {
                L.j[wv][nl + rk] = (uint32_t)j;
                L.m[wv][nl + rk] = m;
            }
            if (nl + n < WAVE) {
                nl += n;
                continue;
            }
            lds_wave_sync();
            tbb_take<MODE>(L.j[wv][lane], L.m[wv][lane], buf, fill, pre, off, cnt, lvl, key0, key1);
            lds_wave_sync();
            if (tied && rk >= first) {
                L.j[wv][rk - first] = (uint32_t)j;
                L.m[wv][rk - first] = m;
            }
            nl = n - first;
        }
    }
    lds_wave_sync();
    if (lane < nl) tbb_take<MODE>(L.j[wv][lane], L.m[wv][lane], buf, fill, pre, off, cnt, lvl, key0, key1);
}

// The nd-th smallest c of the n <= 64 K values v[0..n) (wave-wide, K values per lane in
// registers), and the number lt of values below it: c is fixed bit by bit from the top, bit b
// staying 0 when at least nd values lie at or below the prefix with bits b-1..0 set.  One compare
// and one ballot per bit and register; the result is the same in every lane.
template <int K>
__device__ __forceinline__ void tbb_select(const uint32_t *v, uint32_t n, uint32_t nd, uint32_t &c, uint32_t &lt) {
    const int lane = threadIdx.x & (WAVE - 1);
    uint32_t x[K];
    bool ok[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const uint32_t i = (uint32_t)(lane + q * WAVE);
        ok[q] = i < n;
        x[q] = ok[q] ? v[i] : 0u;
    }
    uint32_t p = 0u;
    for (int b = 31; b >= 0; --b) {
        const uint32_t thr = p | ((1u << b) - 1u);
        uint32_t le = 0u;
#pragma unroll
        for (int q = 0; q < K; ++q) le += (uint32_t)__popcll(__ballot(ok[q] && x[q] <= thr));
        if (le < nd) p |= 1u << b;
    }
    uint32_t below = 0u;
#pragma unroll
    for (int q = 0; q < K; ++q) below += (uint32_t)__popcll(__ballot(ok[q] && x[q] < p));
    c = p;
    lt = below;
}

__global__ __launch_bounds__(TBB_WG) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_b2_tiebreak(const Blk2 *__restrict__ blocks, const uint4 *__restrict__ recs,
                                                        const int32_t *__restrict__ kk, const uint4 *__restrict__ cut,
                                                        uint32_t key0, uint32_t key1, int32_t *__restrict__ rej_at,
                                                        uint32_t *__restrict__ c_out) {
    constexpr int NT = B2U * B2V;
    constexpr int NWV = TBB_WG / WAVE;
    __shared__ uint4 ct[B2U][B2_N1];   // per row u and y0: tie range [lo, hi) of the row's 8 tiles
    __shared__ uint32_t buf[TBB_BUF];
    __shared__ uint32_t pre[NT];       // leading bits of c found so far
    __shared__ uint32_t need[NT];      // rank of c among the tied uniforms with those bits (1-based)
    __shared__ uint32_t bel[NT];       // tied uniforms below those bits
    __shared__ uint32_t cnt[NT];       // tied uniforms with those bits (0: slot finished or idle)
    __shared__ uint32_t off[NT];       // start of the slot's LDS region
    __shared__ uint32_t fill[NT];
    __shared__ int s_next;             // 0: done, 1: histogram pass, 2: gather pass
    __shared__ TbbList lst;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid >> 6;
    const Blk2 *__restrict__ B = blocks + blockIdx.x;
    const int32_t N = B->n_sims;
    const int32_t my_t = B->tile[lane];   // lane = slot in the set-up and bookkeeping steps
    {
        const uint4 *__restrict__ cs = cut + (size_t)blockIdx.x * B2U * B2_N1;
        for (int i = tid; i < B2U * B2_N1; i += TBB_WG) (&ct[0][0])[i] = cs[i];
    }
    if (wv == 0) {
        bool live = false;
        if (my_t >= 0) {
            const int32_t k = kk[my_t];
            live = k >= 1 && k <= N;   // else c was written with the tie ranges
            if (live) need[lane] = (uint32_t)(k - rej_at[my_t]);
        }
        pre[lane] = 0u;
        bel[lane] = 0u;
        cnt[lane] = live ? 1u : 0u;   // marks the live slots until the first pass counts
        fill[lane] = 0u;
    }
    __syncthreads();
    const uint4 *__restrict__ rb = recs + B->key_base;
    // c of slot s: the need-th smallest of the n uniforms at buf[o..o+n) (wave-wide), written out
    auto finish_rank = [&](int s, uint32_t o, uint32_t n) {
        const int32_t t = B->tile[s];
        const uint32_t nd = need[s];
        if (nd > n) {   // no tie class at lambda (lambda not a value of S)
            if (lane == 0) c_out[t] = 0xFFFFFFFFu;
            return;
        }
        uint32_t c, lt;
        if (n <= (uint32_t)WAVE) tbb_select<1>(buf + o, n, nd, c, lt);
        else if (n <= 2u * WAVE) tbb_select<2>(buf + o, n, nd, c, lt);
        else if (n <= 4u * WAVE) tbb_select<4>(buf + o, n, nd, c, lt);
        else tbb_select<8>(buf + o, n, nd, c, lt);
        if (lane == 0) {
            c_out[t] = c;
            rej_at[t] += (int32_t)(bel[s] + lt);
        }
    };
    tbb_sweep<0>(rb, N, ct, lst, buf, fill, pre, off, cnt, 0, key0, key1);
    __syncthreads();
    for (int s = wv; s < NT; s += NWV) {
        if (cnt[s] == 0u) continue;
        const uint32_t n = fill[s];
        if (n <= (uint32_t)TBB_CAPT) {
            finish_rank(s, (uint32_t)(s * TBB_CAPT), n);
            if (lane == 0) cnt[s] = 0u;   // done
        } else if (lane == 0) {
            cnt[s] = n;
        }
    }
    __syncthreads();
    int lvl = 0;
    for (;;) {   // at most 4 rounds: lvl grows by 8 each
        // wave 0: empty the tie ranges of finished slots, decide the next pass
        if (wv == 0) {
            const bool act = cnt[lane] != 0u;
            if (!act) {
                uint8_t *cb = reinterpret_cast<uint8_t *>(&ct[0][0]);
                const int u = lane >> 3, v = lane & 7;
                for (int y0 = 0; y0 < B2_N1; ++y0) cb[(u * B2_N1 + y0) * 16 + 8 + v] = 0;   // hi = 0: empty
            }
            uint32_t mx = cnt[lane], sm = cnt[lane];
            for (int o = 32; o >= 1; o >>= 1) {
                mx = max(mx, __shfl_xor(mx, o));
                sm += __shfl_xor(sm, o);
            }
            if (lane == 0)
                s_next = mx == 0u ? 0 : (lvl > 0 && mx <= (uint32_t)TBB_RANK && sm <= (uint32_t)TBB_BUF ? 2 : 1);
            // gather regions: exclusive prefix of the counts
            const uint32_t mine = act ? cnt[lane] : 0u;
            uint32_t x = mine;
            for (int o = 1; o < WAVE; o <<= 1) {
                const uint32_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            off[lane] = x - mine;
            fill[lane] = 0u;
        }
        for (int i = tid; i < TBB_BUF; i += TBB_WG) buf[i] = 0u;
        __syncthreads();
        const int next = s_next;
        if (next == 0) break;
        if (next == 2) {
            tbb_sweep<2>(rb, N, ct, lst, buf, fill, pre, off, cnt, lvl, key0, key1);
            __syncthreads();
            for (int s = wv; s < NT; s += NWV)
                if (cnt[s] != 0u) finish_rank(s, off[s], cnt[s]);
            break;
        }
        // histogram of the next 8 bits of the uniforms matching the lvl bits known
        tbb_sweep<1>(rb, N, ct, lst, buf, fill, pre, off, cnt, lvl, key0, key1);
        __syncthreads();
        // per active slot (one wave each): the bin holding the need-th uniform
        for (int s = wv; s < NT; s += NWV) {
            if (cnt[s] == 0u) continue;
            const uint32_t *h = buf + s * 256;
            const uint32_t hv[4] = {h[4 * lane], h[4 * lane + 1], h[4 * lane + 2], h[4 * lane + 3]};
            const uint32_t loc = hv[0] + hv[1] + hv[2] + hv[3];
            uint32_t x = loc;
            for (int o = 1; o < WAVE; o <<= 1) {
                const uint32_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            const uint32_t nd = need[s];
            uint32_t run = x - loc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (run < nd && run + hv[q] >= nd) {
                    pre[s] = (pre[s] << 8) | (uint32_t)(4 * lane + q);
                    need[s] = nd - run;
                    bel[s] += run;
                    cnt[s] = hv[q];
                }
                run += hv[q];
            }
        }
        __syncthreads();
        lvl += 8;
        if (lvl == 32) {   // every bit known: c = pre, the ties below it counted in bel
            if (wv == 0 && cnt[lane] != 0u) {
                c_out[my_t] = pre[lane];
                rej_at[my_t] += (int32_t)bel[lane];
            }
            break;
        }
    }
}

// lexicographic minimum of (lambda_i, c_i) over the tiles in the null space; workgroup g takes
// the tiles g, g + gridDim, ... (in 1024-tile strides) and writes its minimum to out_v[g], out_c[g].
__global__ __launch_bounds__(1024) void k_min_pair(const double *__restrict__ v, const uint32_t *__restrict__ c,
                                                   const int32_t *__restrict__ in_null, int64_t n,
                                                   double *__restrict__ out_v, uint32_t *__restrict__ out_c) {
    __shared__ double sv[1024];
    __shared__ uint32_t sc[1024];
    double mv = INFINITY;
    uint32_t mc = 0xFFFFFFFFu;
    for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 1024) {
        if (in_null && !in_null[i]) continue;
        const double x = v[i];
        const uint32_t y = c[i];
        if (x < mv || (x == mv && y < mc)) {
            mv = x;
            mc = y;
        }
    }
    sv[threadIdx.x] = mv;
    sc[threadIdx.x] = mc;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double x = sv[threadIdx.x + s];
            const uint32_t y = sc[threadIdx.x + s];
            if (x < sv[threadIdx.x] || (x == sv[threadIdx.x] && y < sc[threadIdx.x])) {
                sv[threadIdx.x] = x;
                sc[threadIdx.x] = y;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out_v[blockIdx.x] = sv[0];
        out_c[blockIdx.x] = sc[0];
    }
}

// min over tiles of lambda*_i, one workgroup.
// min over the tiles in the null space (in_null[i] != 0; every tile when in_null is NULL)
__global__ __launch_bounds__(1024) void k_min(const double *__restrict__ v, const int32_t *__restrict__ in_null,
                                              int64_t n, double *__restrict__ out) {
    __shared__ double sm[1024];
    double m = INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += 1024)
        if (!in_null || in_null[i]) m = fmin(m, v[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

// partial minima: workgroup g takes the tiles g, g + MIN_PARTS, ... (in 1024-tile strides)
__global__ __launch_bounds__(1024) void k_min_part(const double *__restrict__ v, const int32_t *__restrict__ in_null,
                                                   int64_t n, double *__restrict__ part) {
    __shared__ double sm[1024];
    double m = INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 1024)
        if (!in_null || in_null[i]) m = fmin(m, v[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// Score-function gradient (sum over rejections of T(x) - R grad A(theta)) / N, float64;
// also the float64 score sums and int32 counts for the caller's buffers.
__global__ void k_finish(int fam, int n, int d, int score_n, int64_t n_tiles, const double *__restrict__ theta,
                         const int32_t *__restrict__ N, const uint32_t *__restrict__ R,
                         const unsigned long long *__restrict__ sumT,
                         const unsigned long long *__restrict__ sumZfx, int32_t *__restrict__ R_out,
                         int64_t *__restrict__ T_out, double *__restrict__ Z_out,
                         double *__restrict__ grad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const double r = (double)R[t];
    const double inv = 1.0 / (double)N[t];
    if (R_out) R_out[t] = (int32_t)R[t];
    if (fam == FAM_NORMAL) {
        const double z = (double)(long long)sumZfx[t] * (1.0 / 4294967296.0);
        if (Z_out) Z_out[t] = z;
        if (grad) grad[t] = z * inv;
        return;
    }
    if (score_n) {
        // observed sample sizes: sumT[t] = (sum y_a over a, then sum n_a over a)
        for (int a = 0; a < d; ++a) {
            const unsigned long long sy = sumT[t * 2 * d + a], sn = sumT[t * 2 * d + d + a];
            if (T_out) {
                T_out[t * 2 * d + a] = (int64_t)sy;
                T_out[t * 2 * d + d + a] = (int64_t)sn;
            }
            if (grad) {
                const double p = 1.0 / (1.0 + exp(-theta[t * d + a]));
                grad[t * d + a] = ((double)sy - (double)sn * p) * inv;
            }
        }
        return;
    }
    for (int a = 0; a < d; ++a) {
        const unsigned long long s = sumT[t * d + a];
        if (T_out) T_out[t * d + a] = (int64_t)s;
        if (grad) {
            const double th = theta[t * d + a];
            const double p = 1.0 / (1.0 + exp(-th));
            grad[t * d + a] = ((double)s - r * (double)n * p) * inv;
        }
    }
}

__global__ void k_zero(uint32_t *__restrict__ p, int64_t n_words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_words) p[i] = 0u;
}

// ------------------------------------------------------------------------------ launchers
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    const int64_t words = (int64_t)((bytes + 3) / 4);
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, st, (uint32_t *)p,
                       words);
    return hipGetLastError();
}

hipError_t launch_select(const Platten &P, const void *keys, const int32_t *k, double *lam, int32_t *rej_at,
                         hipStream_t st) {
    if (P.design.kind == CSE_HIER4 || P.design.kind == CSE_BASKET4)   // 64-key chunks at 256-byte offsets: float4 loads
        hipLaunchKernelGGL(k_select_f32<true>, dim3((uint32_t)P.n_tiles), dim3(SEL_WG), 0, st,
                           (const float *)keys, P.d_key_off, P.d_key_stride, P.d_N, k, lam, rej_at);
    else if (P.design.kind != CSE_BINOM2_Z)
        hipLaunchKernelGGL(k_select_f32<false>, dim3((uint32_t)P.n_tiles), dim3(SEL_WG), 0, st,
                           (const float *)keys, P.d_key_off, P.d_key_stride, P.d_N, k, lam, rej_at);
    else {   // the 2-arm bracket (launch_b2_bracket) must have run after k was computed
        const Blk2 *blk = (const Blk2 *)P.d_blocks;
        hipLaunchKernelGGL(k_b2_select, dim3((uint32_t)P.n_blocks), dim3(SEL_WG), 0, st, blk, (const uint4 *)keys, k,
                           P.d_b2br, P.d_b2cut, P.d_S_pos, P.d_S_order, P.d_S_group, P.d_S_tbl, lam, rej_at,
                           P.d_b2fb);
        const uint32_t grid = (uint32_t)std::min<int64_t>(P.n_tiles, 1024);
        hipLaunchKernelGGL(k_b2_full, dim3(grid), dim3(SEL_WG), 0, st, (const uint4 *)keys, P.d_key_off,
                           P.d_key_stride, P.d_N, k, P.d_S_tbl, P.d_S_order, P.d_S_group, P.d_b2fb, lam, rej_at);
    }
    return hipGetLastError();
}

hipError_t launch_h4_bracket(const Platten &P, const float *keys, const int32_t *k, double *lam, int32_t *rej_at,
                             hipStream_t st) {
    if (P.n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_h4_bracket, dim3((uint32_t)P.n_tiles), dim3(SEL_WG), 0, st, keys, P.d_key_off,
                       P.d_key_stride, P.d_N, k, P.h4_margin, P.h4_maxs, P.h4_tot, P.d_h4brk, P.d_h4below,
                       P.d_h4cnt, P.d_h4cand, lam, rej_at);
    return hipGetLastError();
}

hipError_t launch_h4_select(const Platten &P, uint64_t seed, const int32_t *k, double *lam, int32_t *rej_at,
                            hipStream_t st) {
    hipError_t e = launch_zero(P.d_h4fb, sizeof(uint32_t), st);   // the regenerated tiles' list starts empty
    if (e != hipSuccess || P.n_tiles == 0) return e;
    hipLaunchKernelGGL(k_h4_select, dim3((uint32_t)P.n_tiles), dim3(SEL_WG), 0, st, P.d_N, k, P.d_h4below, P.d_h4cnt,
                       P.d_h4cand, P.h4_maxs, P.h4_caps, P.h4_tot, P.d_tileT, P.d_cfg, P.d_h4tbl, (uint32_t)seed,
                       (uint32_t)(seed >> 32), P.d_h4fb, lam, rej_at);
    return hipGetLastError();
}

// 2-arm calibration: brackets and cut points from k (independent of the simulation); resets the
// list of tiles left to the exact full pass.
hipError_t launch_b2_bracket(const Platten &P, const int32_t *k, hipStream_t st) {
    hipLaunchKernelGGL(k_b2_bracket, dim3((uint32_t)P.n_blocks), dim3(WAVE), 0, st, (const Blk2 *)P.d_blocks, k,
                       P.d_gstart, P.d_gcut, P.n_groups, P.d_b2br, P.d_b2cut, P.d_b2fb, P.b2_margin);
    return hipGetLastError();
}

hipError_t launch_tiebreak(const Platten &P, uint64_t seed, const int32_t *k, const double *lam, int32_t *rej_at,
                           uint32_t *c_tile, hipStream_t st) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const dim3 grid((uint32_t)P.n_tiles), blk(SEL_WG);
    if (P.design.kind == CSE_BINOM2_Z) {   // one workgroup per batch of 64 tiles
        if (P.n_blocks > 0) {
            const Blk2 *blk2 = (const Blk2 *)P.d_blocks;
            hipLaunchKernelGGL(k_b2_tiecut, dim3((uint32_t)P.n_blocks), dim3(WAVE), 0, st, blk2, k, lam, P.d_S_tbl,
                               P.d_S_order, P.d_gstart, P.d_gcut, P.n_groups, P.d_b2cut, c_tile);
            hipLaunchKernelGGL(k_b2_tiebreak, dim3((uint32_t)P.n_blocks), dim3(TBB_WG), 0, st, blk2,
                               (const uint4 *)P.d_keys, k, P.d_b2cut, k0, k1, rej_at, c_tile);
        }
    } else if (P.design.kind == CSE_HIER4 || P.design.kind == CSE_BASKET4) {   // 64-key chunks at 256-byte offsets
        hipLaunchKernelGGL(k_tiebreak<TB_F32V4>, grid, blk, 0, st, P.d_keys, P.d_key_off, P.d_key_stride, P.d_N, k,
                           lam, k0, k1, rej_at, c_tile);
    } else {
        hipLaunchKernelGGL(k_tiebreak<TB_F32>, grid, blk, 0, st, P.d_keys, P.d_key_off, P.d_key_stride, P.d_N, k,
                           lam, k0, k1, rej_at, c_tile);
    }
    return hipGetLastError();
}

hipError_t launch_min_pair(const Platten &P, const double *v, const uint32_t *c, const int32_t *in_null, int64_t n,
                           double *out_v, uint32_t *out_c, hipStream_t st) {
    // large inputs: MIN_PARTS partial minima first (values, then their c in the second half of
    // the partial buffer), then one workgroup over them
    if (n > 64 * 1024 && P.d_minpart) {
        double *pv = P.d_minpart;
        uint32_t *pc = reinterpret_cast<uint32_t *>(P.d_minpart + MIN_PARTS);
        hipLaunchKernelGGL(k_min_pair, dim3(MIN_PARTS), dim3(1024), 0, st, v, c, in_null, n, pv, pc);
        hipLaunchKernelGGL(k_min_pair, dim3(1), dim3(1024), 0, st, (const double *)pv, (const uint32_t *)pc,
                           (const int32_t *)nullptr, (int64_t)MIN_PARTS, out_v, out_c);
    } else {
        hipLaunchKernelGGL(k_min_pair, dim3(1), dim3(1024), 0, st, v, c, in_null, n, out_v, out_c);
    }
    return hipGetLastError();
}

hipError_t launch_min(const Platten &P, const double *v, const int32_t *in_null, int64_t n, double *out,
                      hipStream_t st) {
    // large inputs: MIN_PARTS workgroups of partial minima first, then one workgroup over them
    if (n > 64 * 1024 && P.d_minpart) {
        hipLaunchKernelGGL(k_min_part, dim3(MIN_PARTS), dim3(1024), 0, st, v, in_null, n, P.d_minpart);
        hipLaunchKernelGGL(k_min, dim3(1), dim3(1024), 0, st, (const double *)P.d_minpart, (const int32_t *)nullptr,
                           (int64_t)MIN_PARTS, out);
    } else {
        hipLaunchKernelGGL(k_min, dim3(1), dim3(1024), 0, st, v, in_null, n, out);
    }
    return hipGetLastError();
}

hipError_t launch_finish(const Platten &P, const uint32_t *R, const unsigned long long *sumT,
                         const unsigned long long *sumZfx, int32_t *R_out, int64_t *T_out,
                         double *Z_out, double *grad, hipStream_t st) {
    const int64_t grid = (P.n_tiles + 255) / 256;
    hipLaunchKernelGGL(k_finish, dim3((uint32_t)grid), dim3(256), 0, st, P.family, P.n_per_arm, P.d,
                       P.design.kind == CSE_PHASE23 ? 1 : 0, P.n_tiles, P.d_theta, P.d_N, R, sumT, sumZfx, R_out, T_out, Z_out, grad);
    return hipGetLastError();
}

}  // namespace cse
