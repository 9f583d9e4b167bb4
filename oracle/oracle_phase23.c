/*
 * CPU ORACLE -- test infrastructure only (see oracle_sim.c for the conventions).
 *
 * Phase II/III Bayesian selection design (Section 10.2 and its appendix on the design):
 * four Bernoulli arms (arm 0 control), decisions from the hierarchical model of Section 10.1
 * (posterior in oracle_hier.c, here with per-arm sample sizes).  The paper states the protocol
 * but not how p_best and p_success are computed, nor some allocation details.  Reading:
 *
 *  Phase II.  50 patients per arm, then looks after 200, 300, 400 randomised patients.  After
 *    a look without selection the next 100 patients are split evenly over the remaining arms
 *    (control included); the remainder of the division is discarded.
 *  At look t (1..3), for every active treatment arm i:
 *    p_best_i  = P(theta_i is the largest of the four) under independent Gaussian marginals
 *                moment-matched to the posterior node mixture, by 16-point Gauss-Hermite
 *                quadrature of  int phi(t) prod_{k != i} Phi((m_i + s_i t - m_k) / s_k) dt;
 *    p_succ_i  = probability, under a Gaussian predictive, that adding m patients to arm i and
 *                to control (m = 200) yields a final posterior with P(theta_i > theta_0) > 0.95:
 *                d = theta_i - theta_0 ~ N(md, vd) (mixture moments); the added data estimate d
 *                with variance V = 1/(m ph_i (1 - ph_i)) + 1/(m ph_0 (1 - ph_0)),
 *                ph_a = expit(mean_a); the final posterior has variance vf = vd V / (vd + V) and
 *                a mean with predictive law N(md, (vd / (vd + V))^2 (vd + V)), so
 *                p_succ = Phi((md - z95 sqrt(vf)) / (vd / sqrt(vd + V))), z95 = Phi^{-1}(0.95).
 *    If some active arm has p_succ > 0.70 (0.60 at look 3), the active arm with the largest
 *    p_best among those arms is selected (ties: lowest index; arms with equal counts and
 *    sizes have equal posteriors by exchangeability and so tie exactly, whatever rounding
 *    their computed p_best carries).  Otherwise, at looks 1 and 2,
 *    active arms with p_best < 0.15 are dropped (stop for futility if none remains); at look 3
 *    the trial stops for futility.
 *  Phase III.  100 more patients on the selected arm s and on control, then an interim:
 *    P(theta_s > theta_0) > 0.95 -> success (rejection of H_s);  else p_succ_s with m = 100
 *    below 0.20 -> futility;  else 100 more each and the final analysis, which rejects H_s when
 *    P(theta_s > theta_0) > 1 - lambda.
 *  Embedding (Section 9): patient j of arm a uses word a * 350 + j of the simulation's stream
 *    (at most 350 patients per arm), response iff word < T(theta_a).
 *  Calibration statistic for a tile with null configuration b (bit i-1 set when H_i is true):
 *    S = -inf if s is in b and the trial succeeded at the Phase III interim;
 *    S = 1 - P_final(theta_s > theta_0) (summed as a complement) if s is in b and the final
 *        analysis was reached;  S = +inf otherwise.  A false rejection at lambda is S < lambda.
 *  Score: the observed sample sizes and counts, T_a = y_a, grad A_a = n_a expit(theta_a).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define D 4
#define NMAX_ARM 350

uint32_t orc_bern_threshold(double theta);
uint32_t orc_word(uint64_t seed, uint32_t sim, uint32_t w);
void orc_hier4_summary(const int32_t *y, const int32_t *n, double *out, double *diag_mode,
                       double *diag_logw);

static double Phi(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }
static double expit(double x) { return 1.0 / (1.0 + exp(-x)); }

/* ------------------------------------------------------------------ Gauss-Hermite rule
 * 16-point rule for int e^{-x^2} f(x) dx: nodes are the zeros of the Hermite polynomial
 * H_16, weights 2^{n-1} n! sqrt(pi) / (n^2 H_{n-1}(x)^2).  Computed with the orthonormal
 * recurrence h_{k+1} = x sqrt(2/(k+1)) h_k - sqrt(k/(k+1)) h_{k-1}, h_0 = pi^{-1/4}
 * (so the weight is 1 / (n h_{n-1}(x)^2)); zeros bracketed on a fine grid, then bisected. */
#define GH_N 16
static double hermite_orth(int n, double x, double *hnm1) {
    double h0 = pow(acos(-1.0), -0.25), h1 = sqrt(2.0) * x * h0;
    if (n == 0) return h0;
    for (int k = 1; k < n; ++k) {
        double h2 = x * sqrt(2.0 / (k + 1)) * h1 - sqrt((double)k / (k + 1)) * h0;
        h0 = h1;
        h1 = h2;
    }
    *hnm1 = h0;
    return h1;
}

static void gh16_compute(double *x, double *w) {
    int found = 0;
    double prev_x = -8.0, dummy;
    double prev_f = hermite_orth(GH_N, prev_x, &dummy);
    for (int g = 1; g <= 16000 && found < GH_N; ++g) {
        double cx = -8.0 + 16.0 * g / 16000.0, cf = hermite_orth(GH_N, cx, &dummy);
        if ((prev_f < 0) != (cf < 0)) {
            double lo = prev_x, hi = cx, flo = prev_f;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi), fm = hermite_orth(GH_N, mid, &dummy);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
            }
            double r = 0.5 * (lo + hi), hm1;
            hermite_orth(GH_N, r, &hm1);
            x[found] = r;
            w[found] = 1.0 / (GH_N * hm1 * hm1);
            ++found;
        }
        prev_x = cx;
        prev_f = cf;
    }
}

static double g_gx[GH_N], g_gw[GH_N], g_z95;
static int g_consts = 0;

static void init_consts(void) {
    if (g_consts) return;
    gh16_compute(g_gx, g_gw);
    /* z95 = Phi^{-1}(0.95) by bisection on Phi */
    double lo = 0.0, hi = 5.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (Phi(mid) < 0.95) lo = mid; else hi = mid;
    }
    g_z95 = 0.5 * (lo + hi);
    g_consts = 1;
}

void orc_gh16(double *x, double *w) {
    init_consts();
    memcpy(x, g_gx, sizeof g_gx);
    memcpy(w, g_gw, sizeof g_gw);
}

double orc_z95(void) {
    init_consts();
    return g_z95;
}

/* p_best for all four arms from marginal means m[4] and variances v[4]. */
void orc_pbest(const double *m, const double *v, double *pb) {
    init_consts();
    const double *gx = g_gx, *gw = g_gw;
    for (int i = 0; i < D; ++i) {
        double acc = 0.0;
        for (int g = 0; g < GH_N; ++g) {
            double t = m[i] + sqrt(2.0 * v[i]) * gx[g];   /* theta_i at the node */
            double prod = 1.0;
            for (int k = 0; k < D; ++k)
                if (k != i) prod *= Phi((t - m[k]) / sqrt(v[k]));
            acc += gw[g] * prod;
        }
        pb[i] = acc / sqrt(acos(-1.0));
    }
}

/* p_succ for a difference d ~ N(md, vd), control / arm posterior means m0, mi, m added per arm. */
double orc_psucc(double md, double vd, double m0, double mi, int m_add) {
    double p0 = expit(m0), pi = expit(mi);
    double V = 1.0 / (m_add * pi * (1.0 - pi)) + 1.0 / (m_add * p0 * (1.0 - p0));
    double vf = vd * V / (vd + V);
    double sd_mean = vd / sqrt(vd + V);
    return Phi((md - orc_z95() * sqrt(vf)) / sd_mean);
}

/* ------------------------------------------------------------------ the trial */
typedef struct {
    int32_t n[D], y[D];
    uint32_t T[D];
    uint64_t seed;
    uint32_t k;
} trial;

static void add_patients(trial *t, int a, int m) {
    for (int j = t->n[a]; j < t->n[a] + m; ++j)
        if (orc_word(t->seed, t->k, (uint32_t)(a * NMAX_ARM + j)) < t->T[a]) t->y[a] += 1;
    t->n[a] += m;
}

/* Outcome codes of one simulated trial. */
enum { OUT_FUTILITY_P2 = 0, OUT_FUTILITY_P3 = 1, OUT_EARLY_SUCCESS = 2, OUT_FINAL = 3 };

/* One simulation: returns S for configuration cfg; writes the outcome, the selected arm
 * (0 if none), the number of looks and the final n, y; trace (if non-NULL) receives per look
 * [n0..n3, y0..y3] (up to 5 looks). */
static double simulate_trial(trial *t, int cfg, int *outcome, int *sel_out, int *looks,
                             int32_t *trace) {
    double mix[20];
    int active[D] = {0, 1, 1, 1};
    int nl = 0;
    int sel = 0;
    const double z_sel[3] = {0.70, 0.70, 0.60};
    for (int a = 0; a < D; ++a) add_patients(t, a, 50);
    for (int look = 0; look < 3 && !sel; ++look) {
        if (trace) { memcpy(trace + 8 * nl, t->n, sizeof t->n); memcpy(trace + 8 * nl + 4, t->y, sizeof t->y); }
        ++nl;
        orc_hier4_summary(t->y, t->n, mix, NULL, NULL);
        const double *mean = mix + 6, *var = mix + 10, *dm = mix + 14, *dv = mix + 17;
        double pb[D];
        orc_pbest(mean, var, pb);
        int best = 0;
        for (int i = 1; i < D; ++i) {
            if (!active[i]) continue;
            double ps = orc_psucc(dm[i - 1], dv[i - 1], mean[0], mean[i], 200);
            /* equal data give equal p_best whatever the rounding: the lower index stays */
            const int same = best && t->y[i] == t->y[best] && t->n[i] == t->n[best];
            if (ps > z_sel[look] && (best == 0 || (pb[i] > pb[best] && !same))) best = i;
        }
        if (best) { sel = best; break; }
        if (look == 2) break;
        int r = 0;
        for (int i = 1; i < D; ++i) {
            if (active[i] && pb[i] < 0.15) active[i] = 0;
            r += active[i];
        }
        if (r == 0) break;
        const int per = 100 / (r + 1);
        add_patients(t, 0, per);
        for (int i = 1; i < D; ++i)
            if (active[i]) add_patients(t, i, per);
    }
    *sel_out = sel;
    if (!sel) {
        *outcome = OUT_FUTILITY_P2;
        *looks = nl;
        return INFINITY;
    }
    const int in_b = (cfg >> (sel - 1)) & 1;
    add_patients(t, 0, 100);
    add_patients(t, sel, 100);
    if (trace) { memcpy(trace + 8 * nl, t->n, sizeof t->n); memcpy(trace + 8 * nl + 4, t->y, sizeof t->y); }
    ++nl;
    orc_hier4_summary(t->y, t->n, mix, NULL, NULL);
    if (mix[sel - 1] > 0.95) {
        *outcome = OUT_EARLY_SUCCESS;
        *looks = nl;
        return in_b ? -INFINITY : INFINITY;
    }
    if (orc_psucc(mix[14 + sel - 1], mix[17 + sel - 1], mix[6], mix[6 + sel], 100) < 0.20) {
        *outcome = OUT_FUTILITY_P3;
        *looks = nl;
        return INFINITY;
    }
    add_patients(t, 0, 100);
    add_patients(t, sel, 100);
    if (trace) { memcpy(trace + 8 * nl, t->n, sizeof t->n); memcpy(trace + 8 * nl + 4, t->y, sizeof t->y); }
    ++nl;
    orc_hier4_summary(t->y, t->n, mix, NULL, NULL);
    *outcome = OUT_FINAL;
    *looks = nl;
    return in_b ? mix[3 + sel - 1] : INFINITY;
}

/* Tiles (box centre theta[4], configuration cfg).  Per tile: R = #{S < lambda},
 * sumY[4] / sumN[4] = sums of the observed counts and sample sizes over those simulations;
 * optional per simulation: S [tile][stride], info [tile][stride][11] = outcome, selected arm,
 * looks, n[4], y[4]; trace [tile][stride][5][8]. */
void orc_phase23_sim(int64_t n_tiles, const double *theta, const int32_t *cfg, const int32_t *sims,
                     uint64_t seed, double lambda, int32_t *R, int64_t *sumY, int64_t *sumN,
                     double *S, int64_t stride, int32_t *info, int32_t *trace) {
    for (int64_t tt = 0; tt < n_tiles; ++tt) {
        trial base;
        for (int a = 0; a < D; ++a) base.T[a] = orc_bern_threshold(theta[tt * D + a]);
        base.seed = seed;
        int32_t r = 0;
        int64_t sy[D] = {0, 0, 0, 0}, sn[D] = {0, 0, 0, 0};
        for (int32_t k = 0; k < sims[tt]; ++k) {
            trial t = base;
            memset(t.n, 0, sizeof t.n);
            memset(t.y, 0, sizeof t.y);
            t.k = (uint32_t)k;
            int outcome, sel, looks;
            int32_t *tr = trace ? trace + (tt * stride + k) * 40 : NULL;
            if (tr) memset(tr, 0xff, 40 * sizeof(int32_t));
            double s = simulate_trial(&t, cfg[tt], &outcome, &sel, &looks, tr);
            if (s < lambda) {
                r += 1;
                for (int a = 0; a < D; ++a) { sy[a] += t.y[a]; sn[a] += t.n[a]; }
            }
            if (S) S[tt * stride + k] = s;
            if (info) {
                int32_t *f = info + (tt * stride + k) * 11;
                f[0] = outcome;
                f[1] = sel;
                f[2] = looks;
                for (int a = 0; a < D; ++a) { f[3 + a] = t.n[a]; f[7 + a] = t.y[a]; }
            }
        }
        R[tt] = r;
        for (int a = 0; a < D; ++a) {
            if (sumY) sumY[tt * D + a] = sy[a];
            if (sumN) sumN[tt * D + a] = sn[a];
        }
    }
}
