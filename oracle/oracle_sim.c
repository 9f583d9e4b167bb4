/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously correct FP64 implementation of the Monte Carlo part of
 * Continuous Simulation Extension (Yang, Thompson & Sklar, "Guarantees for
 * Comprehensive Simulation Assessment of Statistical Methods").  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * code.  It shares nothing with the HIP library: not a header, not a table,
 * not a constant generator.
 *
 * Conventions (the stream layout and the draw rules; the HIP side implements
 * the same published definitions in its own code):
 *   - Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, Section 3.3): a
 *     10-round Feistel-like bijection on four 32-bit words keyed by two words.
 *   - word(seed, k, w) = Philox4x32-10(key = (seed lo, seed hi),
 *                                      ctr = (w / 4, k, 0, 0))[w mod 4].
 *     Simulation k draws the same words at every tile (common random numbers;
 *     allowed because each tile's own simulations stay i.i.d., Section 7.3).
 *   - Bernoulli(expit(theta)) draw from word u: success iff u < T(theta) with
 *     T(theta) = round(2^32 / (1 + exp(-theta))) clamped to [0, 2^32 - 1].
 *     Arm a, patient j uses word a * n + j (the i.i.d. embedding of Section 9).
 *   - Normal draw (z-test): u_i = ((word_i >> 9) + 1/2) * 2^-23 for words 0, 1;
 *     Z = sqrt(-2 ln u_0) * cos(2 pi u_1) (Box & Muller, 1958).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- Philox */

/* One Philox4x32 round with the multipliers and key schedule of Salmon et al. */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    uint64_t p0 = M0 * (uint64_t)c[0];
    uint64_t p1 = M1 * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {            /* Weyl key bump between rounds */
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

uint32_t orc_word(uint64_t seed, uint32_t sim, uint32_t w) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {w / 4u, sim, 0u, 0u};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[w % 4u];
}

/* Adjoined uniform of the randomised test: first word of the block at counter (0, sim, 1, 0).
 * Data words use counter word 2 = 0, so this stream is disjoint from them, and like them it does
 * not depend on the tile (common random numbers). */
void orc_tiebreak_u(uint64_t seed, int64_t n, uint32_t *out) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t k = 0; k < n; ++k) {
        uint32_t ctr[4] = {0u, (uint32_t)k, 1u, 0u};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        out[k] = o[0];
    }
}

/* ------------------------------------------------------- draw conventions */

uint32_t orc_bern_threshold(double theta) {
    double p = 1.0 / (1.0 + exp(-theta));
    double t = floor(p * 4294967296.0 + 0.5);
    if (t < 0.0) t = 0.0;
    if (t > 4294967295.0) t = 4294967295.0;
    return (uint32_t)t;
}

double orc_unit(uint32_t word) { return ((double)(word >> 9) + 0.5) * (1.0 / 8388608.0); }

double orc_box_muller(uint32_t w0, uint32_t w1) {
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = orc_unit(w0), u1 = orc_unit(w1);
    return sqrt(-2.0 * log(u0)) * cos(two_pi * u1);
}

/* ------------------------------------------------------------- z-test (1-D)
 * X ~ N(theta, 1); reject H0: theta <= 0 when X > cut (Section 4.2).
 * Calibration statistic S = -X, rejection S < lambda (Section 7).
 * Score of the normal location family: T(x) - grad A(theta) = x - theta = Z.
 * Outputs per tile: R (rejections at `cut`), sum over rejections of Z, and
 * optionally S for every simulation (row stride s_stride).
 */
void orc_ztest1(int64_t n_tiles, const double *theta, const int32_t *sims, uint64_t seed,
                double cut, int32_t *R, double *sumZ, double *S, int64_t s_stride) {
    for (int64_t i = 0; i < n_tiles; ++i) {
        int32_t r = 0;
        double sz = 0.0;
        for (int32_t k = 0; k < sims[i]; ++k) {
            double z = orc_box_muller(orc_word(seed, (uint32_t)k, 0), orc_word(seed, (uint32_t)k, 1));
            double x = theta[i] + z;
            if (x > cut) { r += 1; sz += z; }
            if (S) S[i * s_stride + k] = -x;
        }
        R[i] = r;
        if (sumZ) sumZ[i] = sz;
    }
}

/* ------------------------------------------------- two-proportion pooled z
 * Arm 0 control, arm 1 treatment, n patients each, H0: theta1 <= theta0.
 * z = (y1/n - y0/n) / sqrt(pbar (1 - pbar) 2 / n), pbar = (y0 + y1) / (2 n);
 * z = 0 when pbar is 0 or 1 (no information, never rejects).
 */
double orc_pooled_z(int y0, int y1, int n) {
    double pbar = (double)(y0 + y1) / (2.0 * n);
    if (pbar <= 0.0 || pbar >= 1.0) return 0.0;
    double se = sqrt(pbar * (1.0 - pbar) * 2.0 / n);
    return ((double)y1 / n - (double)y0 / n) / se;
}

/* 2-arm binomial design.  theta is [n_tiles][2] (logits of arm 0, arm 1).
 * Per tile: R = #{z > cut}; sumT[a] = sum over rejections of y_a (the
 * sufficient statistic T(x) of Example 1); optionally S = -z per simulation.
 */
void orc_binom2(int64_t n_tiles, const double *theta, const int32_t *sims, uint64_t seed,
                int n, double cut, int32_t *R, int64_t *sumT, double *S, int64_t s_stride) {
    for (int64_t i = 0; i < n_tiles; ++i) {
        uint32_t t0 = orc_bern_threshold(theta[2 * i + 0]);
        uint32_t t1 = orc_bern_threshold(theta[2 * i + 1]);
        int32_t r = 0;
        int64_t s0 = 0, s1 = 0;
        for (int32_t k = 0; k < sims[i]; ++k) {
            int y0 = 0, y1 = 0;
            for (int j = 0; j < n; ++j) {
                if (orc_word(seed, (uint32_t)k, (uint32_t)(0 * n + j)) < t0) y0 += 1;
                if (orc_word(seed, (uint32_t)k, (uint32_t)(1 * n + j)) < t1) y1 += 1;
            }
            double z = orc_pooled_z(y0, y1, n);
            if (z > cut) { r += 1; s0 += y0; s1 += y1; }
            if (S) S[i * s_stride + k] = -z;
        }
        R[i] = r;
        if (sumT) { sumT[2 * i] = s0; sumT[2 * i + 1] = s1; }
    }
}

/* Per-simulation binomial counts of a d-arm design (arm a uses words a*n..a*n+n-1):
 * Y[k][a] for k < sims.  Used by the tests to pin the draw rule. */
void orc_arm_counts(int d, const double *theta, int32_t sims, uint64_t seed, int n, int32_t *Y) {
    for (int32_t k = 0; k < sims; ++k)
        for (int a = 0; a < d; ++a) {
            uint32_t t = orc_bern_threshold(theta[a]);
            int y = 0;
            for (int j = 0; j < n; ++j)
                if (orc_word(seed, (uint32_t)k, (uint32_t)(a * n + j)) < t) y += 1;
            Y[(int64_t)k * d + a] = y;
        }
}
