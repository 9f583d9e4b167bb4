// k_phase23.hip -- the Phase II/III Bayesian selection design (Section 10.2 and the design
// appendix), one simulated trial per lane, decisions from the hierarchical posterior of
// hier_post.hpp (float64) at every look.
//
// Protocol (the reading of the appendix):
//   Phase II: 50 patients per arm; looks after 200, 300 and 400 randomised patients.  At each
//   look, for every active treatment arm i: p_best_i = P(theta_i is the largest of the four)
//   under independent normal marginals moment-matched to the posterior mixture (16-point
//   Gauss-Hermite), and p_succ_i = probability under a Gaussian predictive that adding 200
//   patients to arm i and to control gives P(theta_i > theta_0) > 0.95 at the end.  If some
//   active arm has p_succ > 0.70 (0.60 at the third look) the one with the largest p_best among
//   them is selected (ties: lowest index); otherwise, at looks 1-2, arms with p_best < 0.15 are
//   dropped (futility when none remains) and the next 100 patients are split evenly over the
//   remaining arms and control, the remainder discarded; at look 3 the trial stops.
//   Phase III: 100 + 100 on the selected arm s and control, interim: success if
//   P(theta_s > theta_0) > 0.95, futility if p_succ_s (100 added) < 0.20; else 100 + 100 more and
//   the final analysis.
//   Embedding (Section 9): patient j of arm a draws word a * 350 + j of the simulation's stream.
//   Statistic of a tile with null configuration b: -inf for an early success with s in b,
//   1 - P_final(theta_s > theta_0) for a final analysis with s in b, +inf otherwise; the
//   design's rule at lambda rejects (falsely) when S < lambda.
//
// Scheduling: a persistent grid; each wave pops items (tile, simulation range) from a global
// queue.  Every lane runs its own trial as a state machine, one posterior per step, and takes
// the next simulation (from the wave's current item, or the next item) as soon as its trial
// ends, so lanes whose trials stop early do not wait for long ones.  The first look always has
// 50 patients per arm, so its decision is precomputed per outcome (51^4 bytes, the same decision
// code run once per outcome when the platten is created).  Looks compute only the normal tails
// they use (none in Phase II, the selected arm's in Phase III).  Per trial: the key S is
// stored, and a rejection at the fixed lambda adds to the tile's R and to its sums of the
// observed counts and sample sizes (integer atomics: exact, order-independent).
#include <math.h>

#include "cse_internal.h"
#include "hier_post.hpp"
#include "kernels.h"
#include "philox.hpp"

namespace cse {

namespace {

constexpr int P23_NMAX = 350;   // embedded patients per arm

// Add m patients to arm a (patients n .. n+m-1): count responses among their words.
__device__ __forceinline__ void p23_draw(int a, int m, uint32_t T, uint32_t k, uint32_t key0,
                                         uint32_t key1, int &n, int &y) {
    if (m <= 0) return;
    const uint32_t w0 = (uint32_t)(a * P23_NMAX + n), w1 = w0 + (uint32_t)m;   // [w0, w1)
    int cnt = 0;
    for (uint32_t b = w0 >> 2; b <= (w1 - 1) >> 2; ++b) {
        const u32x4 w = philox_block(b, k, key0, key1);
        const uint32_t base = b << 2;
        cnt += (base + 0 >= w0 && base + 0 < w1 && w.x < T) ? 1 : 0;
        cnt += (base + 1 >= w0 && base + 1 < w1 && w.y < T) ? 1 : 0;
        cnt += (base + 2 >= w0 && base + 2 < w1 && w.z < T) ? 1 : 0;
        cnt += (base + 3 >= w0 && base + 3 < w1 && w.w < T) ? 1 : 0;
    }
    n += m;
    y += cnt;
}

__device__ __forceinline__ double p23_Phi(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

// p_succ for d ~ N(md, vd), control / arm posterior means m0, mi, m_add patients per arm.
__device__ __forceinline__ double p23_psucc(double md, double vd, double m0, double mi, double m_add,
                                            double z95) {
    const double p0 = hp_expit(m0), pi = hp_expit(mi);
    const double V = 1.0 / (m_add * pi * (1.0 - pi)) + 1.0 / (m_add * p0 * (1.0 - p0));
    const double vf = vd * V / (vd + V);
    const double sd_mean = vd / sqrt(vd + V);
    return p23_Phi((md - z95 * sqrt(vf)) / sd_mean);
}

// v[i] for a run-time i in 0..3 without dynamic register indexing.
template <class T>
__device__ __forceinline__ T pick4(const T (&v)[4], int i) {
    return i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
}
template <class T>
__device__ __forceinline__ T pick3(const T (&v)[3], int i) {
    return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]);
}

// Pairs of treatment arms with equal counts and sizes (bit 0: arms 1, 2; bit 1: 1, 3; bit 2: 2, 3).
__device__ __forceinline__ int p23_ties(int y1, int y2, int y3, int n1, int n2, int n3) {
    return ((y1 == y2 && n1 == n2) ? 1 : 0) | ((y1 == y3 && n1 == n3) ? 2 : 0) | ((y2 == y3 && n2 == n3) ? 4 : 0);
}

// Decision at Phase II look `look` (0..2) for the active treatment arms (bit i-1 = arm i):
// code = sel | (active after drops) << 2 | stop << 5, sel = 0 when no arm is selected.  Among
// the arms that qualify the largest p_best wins, the lowest index on ties; arms with equal
// counts and sizes have equal posteriors (exchangeable model), so they tie exactly whatever
// rounding their computed p_best carries: `ties` bit 0 (arms 1, 2), bit 1 (1, 3), bit 2 (2, 3).
__device__ __forceinline__ int p23_phase2(const HierSummary &s, int ties, int look, int active, const double *gh,
                                          double sqrt_pi, double z95) {
    double pb[4] = {0.0, 0.0, 0.0, 0.0};
    double isd[4];   // 1 / (sd * sqrt 2): Phi(z / sd) = erfc(-z isd) / 2
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) isd[kk] = rsq_nr(2.0 * s.var[kk]);
#pragma unroll
    for (int i = 1; i < 4; ++i) {
        const double si = sqrt(2.0 * s.var[i]);
        double acc = 0.0;
        for (int g = 0; g < 16; ++g) {
            const double t = s.mean[i] + si * gh[g];
            double prod = 1.0;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                if (kk != i) prod *= 0.5 * erfc(-(t - s.mean[kk]) * isd[kk]);
            acc += gh[16 + g] * prod;
        }
        pb[i] = acc / sqrt_pi;
    }
    const double thr = (look < 2) ? 0.70 : 0.60;
    int best = 0;
    double pb_best = 0.0;
#pragma unroll
    for (int i = 1; i < 4; ++i) {
        if (!((active >> (i - 1)) & 1)) continue;
        const double ps = p23_psucc(s.mean[i] - s.mean[0], s.dvar[i - 1], s.mean[0], s.mean[i], 200.0, z95);
        const bool same = best != 0 && ((ties >> (best + i - 3)) & 1);   // best < i
        if (ps > thr && (best == 0 || (pb[i] > pb_best && !same))) {
            best = i;
            pb_best = pb[i];
        }
    }
    if (best) return best | (active << 2);
    if (look == 2) return (active << 2) | (1 << 5);
#pragma unroll
    for (int i = 1; i < 4; ++i)
        if (((active >> (i - 1)) & 1) && pb[i] < 0.15) active &= ~(1 << (i - 1));
    return (active << 2) | ((active == 0 ? 1 : 0) << 5);
}

}  // namespace

// Decision of the first look (50 patients per arm) for every outcome y in {0..50}^4, index
// ((y0 51 + y1) 51 + y2) 51 + y3; the trials take it from here instead of a posterior.
__global__ __launch_bounds__(128) void k_p23_look1(int64_t n_out, uint8_t *__restrict__ tbl,
                                                   const HierNode *__restrict__ nodes,
                                                   const double *__restrict__ gh, double sqrt_pi, double z95) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_out) return;
    int y[4];
    int64_t v = idx;
    for (int a = 3; a >= 0; --a) {
        y[a] = (int)(v % 51);
        v /= 51;
    }
    const double n[4] = {50.0, 50.0, 50.0, 50.0};
    HierSummary s;
    hier_posterior<true, true>(y, n, nodes, s, nullptr, 0);
    tbl[idx] = (uint8_t)p23_phase2(s, p23_ties(y[1], y[2], y[3], 50, 50, 50), 0, 7, gh, sqrt_pi, z95);
}

hipError_t launch_p23_look1(const Platten &P, hipStream_t st) {
    const int64_t n_out = 51LL * 51 * 51 * 51;
    hipLaunchKernelGGL(k_p23_look1, dim3((uint32_t)((n_out + 127) / 128)), dim3(128), 0, st, n_out, P.d_p23look1,
                       P.d_hnodes, P.d_gh, P.p23.sqrt_pi, P.p23.z95);
    return hipGetLastError();
}

// Two waves per SIMD: the float64 posterior keeps about 250 registers live.
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_phase23(P23Args A) {
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    // wave-uniform current item
    int32_t it_tile = -1;
    uint32_t it_k = 0, it_end = 0;
    bool queue_open = true;

    // lane state: busy = a trial in progress; add[a] = patients to enrol on arm a before the
    // next look; look 0..2 Phase II, 3 Phase III interim, 4 final analysis
    bool busy = false;
    int32_t tile = 0;
    uint32_t k = 0, T[4] = {0u, 0u, 0u, 0u};
    int cfg = 0, look = 0, sel = 0, active = 0;
    int n[4] = {0, 0, 0, 0}, y[4] = {0, 0, 0, 0}, add[4] = {0, 0, 0, 0};
    int c_trials = 0, c_look2 = 0, c_look3 = 0, c_newton = 0;   // this lane's work (stats counters)

    bool fresh = false, done = false;
    float S = INFINITY;
    // Phase II decision code -> next enrolment (or the end of the trial)
    auto apply = [&](int code) {
        const int s_arm = code & 3;
        if (s_arm) {
            sel = s_arm;
#pragma unroll
            for (int a = 0; a < 4; ++a) add[a] = (a == 0 || a == s_arm) ? 100 : 0;
            look = 3;
        } else if ((code >> 5) & 1) {
            done = true;
        } else {
            active = (code >> 2) & 7;
            const int per = 100 / (__popc(active) + 1);
#pragma unroll
            for (int a = 0; a < 4; ++a) add[a] = (a == 0 || ((active >> (a - 1)) & 1)) ? per : 0;
            look += 1;
        }
    };
    // the trial's result: its key, and the rejection sums when S is below the cut
    auto finish = [&]() {
        if (A.keys) A.keys[A.key_off[tile] + k] = S;
        if (S < A.cut) {
            atomicAdd(&A.R[tile], 1u);
            if (A.sumT)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    atomicAdd(&A.sumT[(int64_t)tile * 8 + a], (unsigned long long)y[a]);
                    atomicAdd(&A.sumT[(int64_t)tile * 8 + 4 + a], (unsigned long long)n[a]);
                }
        }
        busy = false;
        c_trials += 1;
    };

    for (;;) {
        // ---- give idle lanes the next simulations of the wave's item stream and run their first
        // look (a table lookup); a trial that ends there is finished at once and its lane takes
        // another, so that lanes do not sit out the posterior below ----
        for (;;) {
            unsigned long long need = __ballot(!busy);
            while (need) {
                if (it_k >= it_end) {
                    if (!queue_open) break;
                    uint32_t idx = 0;
                    if (lane == 0) idx = atomicAdd(A.counter, 1u);
                    idx = __builtin_amdgcn_readfirstlane(idx);
                    if ((int64_t)idx >= A.n_items) {
                        queue_open = false;
                        break;
                    }
                    const WorkItem W = A.items[idx];
                    it_tile = W.blk;
                    it_k = W.k_begin;
                    it_end = W.k_end;
                    continue;
                }
                const uint32_t avail = it_end - it_k;
                const uint32_t rank = (uint32_t)__popcll(need & below);
                if (((need >> lane) & 1ull) && rank < avail) {
                    busy = true;
                    fresh = true;
                    tile = it_tile;
                    k = it_k + rank;
                    for (int a = 0; a < 4; ++a) {
                        T[a] = A.tileT[(int64_t)tile * 4 + a];
                        n[a] = 0;
                        y[a] = 0;
                    }
                    cfg = A.cfg[tile];
                    look = 0;
                    sel = 0;
                    active = 7;
                }
                const uint32_t asked = (uint32_t)__popcll(need);
                it_k += asked < avail ? asked : avail;
                need = __ballot(!busy);
            }
            if (!__ballot(fresh)) break;   // nobody was given a trial: all lanes busy, or queue drained
            if (fresh) {
                // Phase II opens with 50 patients per arm; the first look's decision is tabulated
                fresh = false;
                done = false;
                S = INFINITY;
#pragma unroll
                for (int a = 0; a < 4; ++a) p23_draw(a, 50, T[a], k, A.key0, A.key1, n[a], y[a]);
                apply(A.look1[((y[0] * 51 + y[1]) * 51 + y[2]) * 51 + y[3]]);
                if (done) finish();
            }
        }
        if (!__ballot(busy)) break;   // queue drained and every trial finished
        if (busy) {
            // ---- enrol the patients of the next look, then one posterior look ----
#pragma unroll
            for (int a = 0; a < 4; ++a) p23_draw(a, add[a], T[a], k, A.key0, A.key1, n[a], y[a]);
            HierSummary s;
            {
                const double nd[4] = {(double)n[0], (double)n[1], (double)n[2], (double)n[3]};
                // tails the wave needs (a uniform mask keeps the branch scalar)
                const int mine = look < 3 ? 0 : 1 << (sel - 1);
                int wneed = 0;
#pragma unroll
                for (int i = 0; i < 3; ++i) wneed |= __ballot((mine >> i) & 1) ? (1 << i) : 0;
                hier_posterior<true, true>(y, nd, A.nodes, s, &c_newton, __builtin_amdgcn_readfirstlane(wneed));
            }
            if (look < 3) c_look2 += 1; else c_look3 += 1;
            if (look < 3) {
                apply(p23_phase2(s, p23_ties(y[1], y[2], y[3], n[1], n[2], n[3]), look, active, A.gh, A.sqrt_pi,
                                 A.z95));
            } else {
                const bool in_b = (cfg >> (sel - 1)) & 1;
                if (look == 3) {
                    // Phase III interim
                    const double ms = pick4(s.mean, sel);
                    if (pick3(s.P, sel - 1) > 0.95) {
                        S = in_b ? -INFINITY : INFINITY;
                        done = true;
                    } else if (p23_psucc(ms - s.mean[0], pick3(s.dvar, sel - 1), s.mean[0], ms, 100.0, A.z95) <
                               0.20) {
                        done = true;
                    } else {
#pragma unroll
                        for (int a = 0; a < 4; ++a) add[a] = (a == 0 || a == sel) ? 100 : 0;
                        look = 4;
                    }
                } else {
                    // final analysis
                    S = in_b ? (float)pick3(s.Sc, sel - 1) : INFINITY;
                    done = true;
                }
            }
            if (done) finish();
        }
    }
    if (A.stats) {
        // one atomic per counter and wave: reduce the lane counters across the wave first
        unsigned long long c[4] = {(unsigned long long)c_trials, (unsigned long long)c_look2,
                                   (unsigned long long)c_look3, (unsigned long long)c_newton};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            for (int off = 32; off >= 1; off >>= 1) c[i] += __shfl_xor(c[i], off);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) atomicAdd(&A.stats[i], c[i]);
    }
}

hipError_t launch_phase23(const Platten &P, uint64_t seed, uint32_t *R, unsigned long long *sumT, float *keys,
                          hipStream_t st) {
    hipError_t e = launch_zero(P.d_queue, sizeof(uint32_t), st);
    if (e != hipSuccess) return e;
    P23Args A = P.p23;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.R = R;
    A.sumT = sumT;
    A.keys = keys;
    A.stats = P.d_p23stats;
    e = launch_zero(P.d_p23stats, 4 * sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_phase23, dim3((uint32_t)P.p23_grid), dim3(WG), 0, st, A);
    return hipGetLastError();
}

// A launch over a caller-made item list (schedule tuning on a sample of tiles); counts only.
hipError_t launch_phase23_items(const Platten &P, uint64_t seed, const WorkItem *items, int64_t n_items, int64_t grid,
                                uint32_t *R, hipStream_t st) {
    hipError_t e = launch_zero(P.d_queue, sizeof(uint32_t), st);
    if (e != hipSuccess) return e;
    P23Args A = P.p23;
    A.items = items;
    A.n_items = n_items;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.R = R;
    A.sumT = nullptr;
    A.keys = nullptr;
    A.stats = nullptr;
    hipLaunchKernelGGL(k_phase23, dim3((uint32_t)grid), dim3(WG), 0, st, A);
    return hipGetLastError();
}

// The plain path: one launch per tile over that tile's own queue items (no other tiles share
// the grid); counts only.
hipError_t launch_phase23_tile(const Platten &P, uint64_t seed, int64_t t, uint32_t *R_tile, hipStream_t st) {
    hipError_t e = launch_zero(P.d_queue, sizeof(uint32_t), st);
    if (e != hipSuccess) return e;
    P23Args A = P.p23;
    const int64_t i0 = P.p23_item_off[t], i1 = P.p23_item_off[t + 1];
    A.items = P.d_p23items + i0;
    A.n_items = i1 - i0;
    A.key0 = (uint32_t)seed;
    A.key1 = (uint32_t)(seed >> 32);
    A.R = R_tile - t;   // the kernel indexes R by tile id
    A.sumT = nullptr;
    A.keys = nullptr;
    A.stats = nullptr;
    hipLaunchKernelGGL(k_phase23, dim3((uint32_t)((A.n_items + 3) / 4)), dim3(WG), 0, st, A);
    return hipGetLastError();
}

}  // namespace cse
