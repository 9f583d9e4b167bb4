/*
 * CPU ORACLE -- test infrastructure only (see oracle_sim.c for the conventions).
 *
 * Four Bernoulli arms (arm 0 control), n patients each, hierarchical model of the
 * Bayesian basket case study (Section 10.1):
 *     theta_i | mu, s2 ~ N(mu, s2),  mu ~ N(-1.34, 100),  s2 ~ InvGamma(0.0005, 0.000005),
 *     y_i ~ Binom(n, expit(theta_i)).
 * The statistic of treatment arm i is P(p_i > p_0 | y) = P(theta_i > theta_0 | y).
 *
 * The paper gives the model but not how its posterior is computed.  Reading used here:
 *   1. mu is integrated out exactly: theta | s2 ~ N(m0 1, Sigma), Sigma = s2 I + 100 11^T, with
 *      Sigma^{-1} and log|Sigma| in closed form (Sherman-Morrison, determinant lemma).
 *   2. For each of 90 nodes s2_j (equally spaced in log s2 over [log 1e-6, log 1e3]), the
 *      conditional posterior of theta is replaced by its Laplace (Gaussian) approximation:
 *      mode by Newton's method, covariance C_j = (-H)^{-1} at the mode.
 *   3. Node weights: Laplace evidence  l(mode) + log|Q| / 2 - log|-H| / 2  (Q = Sigma^{-1}),
 *      plus the log prior density of s2_j, plus the log trapezoid weight in log s2
 *      (ds2 = s2 dlog s2); normalised by log-sum-exp in float64.
 *   4. P_i(y) = sum_j pi_j Phi((mode_i - mode_0) / sd), sd^2 = Var(theta_i - theta_0) under C_j.
 * Property of this reading: at the boundary counts y_i in {0, n} the Gaussian replacing the
 * skewed conditional posterior is very wide, so P_i is not monotone there (it is monotone
 * for interior counts).
 * All float64; the Newton systems and variances by generic 4x4 Gaussian elimination.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define D 4
#define NODES 90

static const double M0 = -1.34, TAU2 = 100.0;
static const double IG_A = 0.0005, IG_B = 0.000005;
static const double LS2_LO = -13.815510557964274, LS2_HI = 6.907755278982137; /* log 1e-6, log 1e3 */

uint32_t orc_bern_threshold(double theta);
uint32_t orc_word(uint64_t seed, uint32_t sim, uint32_t w);

static double softplus(double x) { return x > 0 ? x + log1p(exp(-x)) : log1p(exp(x)); }
static double expit(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Solve A x = b (A is overwritten) by Gaussian elimination with partial pivoting. */
static void solve4(double A[D][D], double b[D], double x[D]) {
    for (int c = 0; c < D; ++c) {
        int p = c;
        for (int r = c + 1; r < D; ++r)
            if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (p != c) {
            for (int j = 0; j < D; ++j) { double t = A[c][j]; A[c][j] = A[p][j]; A[p][j] = t; }
            double t = b[c]; b[c] = b[p]; b[p] = t;
        }
        for (int r = c + 1; r < D; ++r) {
            double f = A[r][c] / A[c][c];
            for (int j = c; j < D; ++j) A[r][j] -= f * A[c][j];
            b[r] -= f * b[c];
        }
    }
    for (int r = D - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < D; ++j) s -= A[r][j] * x[j];
        x[r] = s / A[r][r];
    }
}

/* log det of a symmetric positive definite matrix by elimination (product of pivots). */
static double logdet4(const double M[D][D]) {
    double A[D][D];
    memcpy(A, M, sizeof A);
    double ld = 0.0;
    for (int c = 0; c < D; ++c) {
        int p = c;
        for (int r = c + 1; r < D; ++r)
            if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (p != c)
            for (int j = 0; j < D; ++j) { double t = A[c][j]; A[c][j] = A[p][j]; A[p][j] = t; }
        ld += log(fabs(A[c][c]));
        for (int r = c + 1; r < D; ++r) {
            double f = A[r][c] / A[c][c];
            for (int j = c; j < D; ++j) A[r][j] -= f * A[c][j];
        }
    }
    return ld;
}

static __attribute__((unused)) void inverse4(const double M[D][D], double Inv[D][D]) {
    for (int k = 0; k < D; ++k) {
        double A[D][D], e[D] = {0}, x[D];
        memcpy(A, M, sizeof A);
        e[k] = 1.0;
        solve4(A, e, x);
        for (int r = 0; r < D; ++r) Inv[r][k] = x[r];
    }
}

static double Phi(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

/* Node j: log s2 value and trapezoid weight (in log s2). */
void orc_hier4_node(int j, double *ls2, double *logw) {
    double h = (LS2_HI - LS2_LO) / (NODES - 1);
    *ls2 = LS2_LO + h * j;
    double w = (j == 0 || j == NODES - 1) ? 0.5 * h : h;
    *logw = log(w) + *ls2;   /* ds2 = s2 dlog s2 */
}

/* Posterior of one outcome y (counts out of n per arm).  Outputs P[3] = P(theta_i > theta_0 | y)
 * for i = 1, 2, 3; if diag != NULL also per-node mode [NODES][D], log weight [NODES] and
 * Newton iterations [NODES] (for the tests). */
/* Per-arm sample sizes nv[4].  Outputs P[3], Sc[3] = 1 - P (summed as complements); if
 * mix != NULL the moment-matched mixture summary (see orc_hier4_summary). */
static void posterior_nv(const int32_t *y, const int32_t *nv, double *P, double *Sc, double *mix,
                         double *diag_mode, double *diag_logw, int32_t *diag_iters) {
    double lw[NODES], pr[NODES][3], pc[NODES][3];
    double mode[NODES][D], cdiag[NODES][D], dvar[NODES][3];
    for (int j = 0; j < NODES; ++j) {
        double ls2, logtrap;
        orc_hier4_node(j, &ls2, &logtrap);
        double s2 = exp(ls2);
        /* Q = Sigma^{-1} for Sigma = s2 I + TAU2 11^T, in closed form (Sherman-Morrison):
         * Q = (I - cq 11^T) / s2 with cq = TAU2 / (s2 + D TAU2).  (Inverting Sigma numerically
         * loses ~8 digits: its condition number is (s2 + D TAU2) / s2, ~4e8 at s2 = 1e-6.) */
        double Q[D][D];
        const double cq = TAU2 / (s2 + D * TAU2);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) Q[r][c] = ((r == c ? 1.0 : 0.0) - cq) / s2;
        /* log|Q| = -log|Sigma| = -((D - 1) log s2 + log(s2 + D TAU2)) (matrix determinant lemma) */
        const double logdetQ = -((D - 1) * ls2 + log(s2 + D * TAU2));
        double th[D];
        for (int a = 0; a < D; ++a) th[a] = log((y[a] + 0.5) / (nv[a] - y[a] + 0.5));
        int it = 0;
        double H[D][D];
        for (it = 0; it < 200; ++it) {
            double g[D];
            for (int a = 0; a < D; ++a) {
                double qa = 0.0;
                for (int c = 0; c < D; ++c) qa += Q[a][c] * (th[c] - M0);
                g[a] = y[a] - nv[a] * expit(th[a]) - qa;
            }
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c) {
                    double p = expit(th[r]);
                    H[r][c] = -Q[r][c] - (r == c ? nv[r] * p * (1.0 - p) : 0.0);
                }
            double A[D][D], step[D], rhs[D];
            memcpy(A, H, sizeof A);
            for (int a = 0; a < D; ++a) rhs[a] = g[a];
            solve4(A, rhs, step);                    /* H step = g  ->  theta -= step */
            double mx = 0.0;
            for (int a = 0; a < D; ++a) {
                th[a] -= step[a];
                mx = fmax(mx, fabs(step[a]));
            }
            if (mx < 1e-10) break;   /* rounding floor of the step is ~1e-11 at the smallest s2 */
        }
        /* curvature at the final mode */
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                double p = expit(th[r]);
                H[r][c] = -Q[r][c] - (r == c ? nv[r] * p * (1.0 - p) : 0.0);
            }
        double negH[D][D];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) negH[r][c] = -H[r][c];
        double ll = 0.0, quad = 0.0;
        for (int a = 0; a < D; ++a) ll += y[a] * th[a] - nv[a] * softplus(th[a]);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) quad += (th[r] - M0) * Q[r][c] * (th[c] - M0);
        double lap = ll - 0.5 * quad + 0.5 * logdetQ - 0.5 * logdet4(negH);
        double logprior = IG_A * log(IG_B) - lgamma(IG_A) - (IG_A + 1.0) * ls2 - IG_B / s2;
        lw[j] = lap + logprior + logtrap;
        for (int i = 1; i < D; ++i) {
            /* Var(theta_i - theta_0) = e^T C e = e^T x with (-H) x = e, e = e_i - e_0: solving for
             * x avoids the cancellation in C_ii + C_00 - 2 C_i0 when the arms are tightly linked */
            double A[D][D], e[D] = {0, 0, 0, 0}, x[D];
            memcpy(A, negH, sizeof A);
            e[i] = 1.0;
            e[0] = -1.0;
            solve4(A, e, x);
            double sd = sqrt(x[i] - x[0]);
            pr[j][i - 1] = Phi((th[i] - th[0]) / sd);
            pc[j][i - 1] = Phi(-(th[i] - th[0]) / sd);   /* 1 - Phi(z), no cancellation */
            dvar[j][i - 1] = x[i] - x[0];
        }
        for (int a = 0; a < D; ++a) {
            /* C_aa = e_a^T (-H)^{-1} e_a */
            double A[D][D], e[D] = {0, 0, 0, 0}, x[D];
            memcpy(A, negH, sizeof A);
            e[a] = 1.0;
            solve4(A, e, x);
            cdiag[j][a] = x[a];
            mode[j][a] = th[a];
        }
        if (diag_mode)
            for (int a = 0; a < D; ++a) diag_mode[j * D + a] = th[a];
        if (diag_iters) diag_iters[j] = it;
    }
    double mx = -INFINITY;
    for (int j = 0; j < NODES; ++j) mx = fmax(mx, lw[j]);
    double s = 0.0;
    for (int j = 0; j < NODES; ++j) s += exp(lw[j] - mx);
    double lse = mx + log(s);
    for (int i = 0; i < 3; ++i) P[i] = Sc[i] = 0.0;
    double pj[NODES];
    for (int j = 0; j < NODES; ++j) {
        pj[j] = exp(lw[j] - lse);
        if (diag_logw) diag_logw[j] = lw[j] - lse;
        for (int i = 0; i < 3; ++i) {
            P[i] += pj[j] * pr[j][i];
            Sc[i] += pj[j] * pc[j][i];
        }
    }
    if (!mix) return;
    /* Moment matching of the node mixture (two passes: means, then spreads about them):
     * mean_a = sum_j pi_j mode_ja, var_a = sum_j pi_j (C_j,aa + (mode_ja - mean_a)^2), and the
     * same for the differences d_i = theta_i - theta_0. */
    double mean[D] = {0, 0, 0, 0}, var[D] = {0, 0, 0, 0}, dm[3] = {0, 0, 0}, dv[3] = {0, 0, 0};
    for (int j = 0; j < NODES; ++j)
        for (int a = 0; a < D; ++a) mean[a] += pj[j] * mode[j][a];
    for (int i = 0; i < 3; ++i) dm[i] = mean[i + 1] - mean[0];
    for (int j = 0; j < NODES; ++j) {
        for (int a = 0; a < D; ++a) {
            double e = mode[j][a] - mean[a];
            var[a] += pj[j] * (cdiag[j][a] + e * e);
        }
        for (int i = 0; i < 3; ++i) {
            double e = (mode[j][i + 1] - mode[j][0]) - dm[i];
            dv[i] += pj[j] * (dvar[j][i] + e * e);
        }
    }
    for (int i = 0; i < 3; ++i) { mix[i] = P[i]; mix[3 + i] = Sc[i]; }
    for (int a = 0; a < D; ++a) { mix[6 + a] = mean[a]; mix[10 + a] = var[a]; }
    for (int i = 0; i < 3; ++i) { mix[14 + i] = dm[i]; mix[17 + i] = dv[i]; }
}

static void posterior_full(const int32_t *y, int n, double *P, double *Sc, double *diag_mode,
                           double *diag_logw, int32_t *diag_iters) {
    const int32_t nv[D] = {n, n, n, n};
    posterior_nv(y, nv, P, Sc, NULL, diag_mode, diag_logw, diag_iters);
}

/* Posterior summary with per-arm sample sizes n[4] (counts y[a] out of n[a]):
 * out[0..2] P(theta_i > theta_0), out[3..5] their complements, out[6..9] mixture means of
 * theta_a, out[10..13] mixture variances, out[14..16] means and out[17..19] variances of
 * theta_i - theta_0.  Diagnostics as in orc_hier4_posterior_full when non-NULL. */
void orc_hier4_summary(const int32_t *y, const int32_t *n, double *out, double *diag_mode,
                       double *diag_logw) {
    double P[3], Sc[3];
    posterior_nv(y, n, P, Sc, out, diag_mode, diag_logw, NULL);
}

void orc_hier4_posterior_full(const int32_t *y, int n, double *P, double *diag_mode,
                              double *diag_logw, int32_t *diag_iters) {
    double Sc[3];
    posterior_full(y, n, P, Sc, diag_mode, diag_logw, diag_iters);
}

void orc_hier4_posterior(const int32_t *y, int n, double *P) {
    double Sc[3];
    posterior_full(y, n, P, Sc, NULL, NULL, NULL);
}

/* The design statistic 1 - P_i(y) summed as sum_j pi_j Phi(-z_j): relative precision for
 * small values, which a subtraction 1 - P would lose when P is near 1. */
void orc_hier4_complement(const int32_t *y, int n, double *S) {
    double P[3];
    posterior_full(y, n, P, S, NULL, NULL, NULL);
}

/* The statistics 1 - P_i(y), i = 1..3, for a list of outcome indices
 * idx = ((y0*(n+1)+y1)*(n+1)+y2)*(n+1)+y3. */
void orc_hier4_table(int n, const int64_t *idx, int64_t count, double *out /* [count][3] */) {
    const int64_t m = n + 1;
    for (int64_t t = 0; t < count; ++t) {
        int64_t v = idx[t];
        int32_t y[D];
        for (int a = D - 1; a >= 0; --a) {
            y[a] = (int32_t)(v % m);
            v /= m;
        }
        orc_hier4_complement(y, n, out + 3 * t);
    }
}

/* ------------------------------------------------------------------ simulation
 * Tiles are (box centre theta [4], null configuration b) pairs; simulation k draws arm a,
 * patient j from word a*n + j, as in oracle_sim.c.  For configuration b (bit i-1 set when
 * H_i: theta_i <= theta_0 is true) the statistic is S_b = min_{i in b} (1 - P_i(y)) and the
 * design rejects (a true null, i.e. the FWER event of the configuration) when S_b < cut.
 * Outputs per tile: R, sumT[4] = sum over rejections of y, optional S [tile][stride] and the
 * outcome index of every simulation.  Posteriors are memoised by outcome.
 */
#include <stdlib.h>

static double *g_memo = NULL;
static unsigned char *g_have = NULL;
static int g_memo_n = -1;

static const double *memo_posterior(const int32_t *y, int n) {
    const int64_t m = n + 1;
    if (g_memo_n != n) {
        free(g_memo);
        free(g_have);
        g_memo = (double *)malloc(sizeof(double) * 3 * m * m * m * m);
        g_have = (unsigned char *)calloc((size_t)(m * m * m * m), 1);
        g_memo_n = n;
    }
    int64_t idx = ((y[0] * m + y[1]) * m + y[2]) * m + y[3];
    if (!g_have[idx]) {
        orc_hier4_complement(y, n, g_memo + 3 * idx);
        g_have[idx] = 1;
    }
    return g_memo + 3 * idx;
}

void orc_hier4_sim(int64_t n_tiles, const double *theta, const int32_t *cfg, const int32_t *sims,
                   uint64_t seed, int n, double cut, int32_t *R, int64_t *sumT, double *S,
                   int64_t s_stride, int64_t *outcome) {
    const int64_t m = n + 1;
    for (int64_t t = 0; t < n_tiles; ++t) {
        uint32_t T[D];
        for (int a = 0; a < D; ++a) T[a] = orc_bern_threshold(theta[t * D + a]);
        int32_t r = 0;
        int64_t st[D] = {0, 0, 0, 0};
        for (int32_t k = 0; k < sims[t]; ++k) {
            int32_t y[D];
            for (int a = 0; a < D; ++a) {
                y[a] = 0;
                for (int j = 0; j < n; ++j)
                    if (orc_word(seed, (uint32_t)k, (uint32_t)(a * n + j)) < T[a]) y[a] += 1;
            }
            const double *Sc = memo_posterior(y, n);   /* 1 - P_i(y) */
            double s = INFINITY;
            for (int i = 1; i < D; ++i)
                if ((cfg[t] >> (i - 1)) & 1) s = fmin(s, Sc[i - 1]);
            if (s < cut) {
                r += 1;
                for (int a = 0; a < D; ++a) st[a] += y[a];
            }
            if (S) S[t * s_stride + k] = s;
            if (outcome) outcome[t * s_stride + k] = ((y[0] * m + y[1]) * m + y[2]) * m + y[3];
        }
        R[t] = r;
        if (sumT)
            for (int a = 0; a < D; ++a) sumT[t * D + a] = st[a];
    }
}

/* ------------------------------------------------------------------ basket design
 * Bayesian basket trial (Section 10.1, validation case study): four arms, each against its own
 * fixed standard-of-care rate p_0a (theta_0a = logit p_0a).  The hierarchical model is on the
 * offsets delta_a = theta_a - theta_0a:
 *     delta_a | mu, s2 ~ N(mu, s2),  mu ~ N(-1.34, 100),  s2 ~ InvGamma(0.0005, 0.000005),
 *     y_a ~ Binom(n, expit(theta_a)).
 * In theta the prior has mean -1.34 + theta_0a per arm and the same covariance, so the reading
 * above applies unchanged (90 s2 nodes, Laplace per node, Laplace evidence weights).  The
 * statistic of arm a is P(p_a > p_0a | y) = P(theta_a > theta_0a | y); its complement is
 * summed directly, sum_j pi_j Phi(-(mode_ja - theta_0a) / sqrt(C_j,aa)).
 * All float64, generic 4x4 elimination as above.
 */
void orc_basket_complement(const int32_t *y, int n, const double *theta0, double *Sc) {
    double lw[NODES], pc[NODES][D];
    for (int j = 0; j < NODES; ++j) {
        double ls2, logtrap;
        orc_hier4_node(j, &ls2, &logtrap);
        const double s2 = exp(ls2);
        double Q[D][D];
        const double cq = TAU2 / (s2 + D * TAU2);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) Q[r][c] = ((r == c ? 1.0 : 0.0) - cq) / s2;
        const double logdetQ = -((D - 1) * ls2 + log(s2 + D * TAU2));
        double mean[D], th[D], H[D][D];
        for (int a = 0; a < D; ++a) {
            mean[a] = M0 + theta0[a];
            th[a] = log((y[a] + 0.5) / (n - y[a] + 0.5));
        }
        for (int it = 0; it < 200; ++it) {
            double g[D];
            for (int a = 0; a < D; ++a) {
                double qa = 0.0;
                for (int c = 0; c < D; ++c) qa += Q[a][c] * (th[c] - mean[c]);
                g[a] = y[a] - n * expit(th[a]) - qa;
            }
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c) {
                    const double p = expit(th[r]);
                    H[r][c] = -Q[r][c] - (r == c ? n * p * (1.0 - p) : 0.0);
                }
            double A[D][D], step[D], rhs[D];
            memcpy(A, H, sizeof A);
            for (int a = 0; a < D; ++a) rhs[a] = g[a];
            solve4(A, rhs, step);
            double mx = 0.0;
            for (int a = 0; a < D; ++a) {
                th[a] -= step[a];
                mx = fmax(mx, fabs(step[a]));
            }
            if (mx < 1e-10) break;
        }
        double negH[D][D];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                const double p = expit(th[r]);
                negH[r][c] = Q[r][c] + (r == c ? n * p * (1.0 - p) : 0.0);
            }
        double ll = 0.0, quad = 0.0;
        for (int a = 0; a < D; ++a) ll += y[a] * th[a] - n * softplus(th[a]);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) quad += (th[r] - mean[r]) * Q[r][c] * (th[c] - mean[c]);
        const double lap = ll - 0.5 * quad + 0.5 * logdetQ - 0.5 * logdet4(negH);
        const double logprior = IG_A * log(IG_B) - lgamma(IG_A) - (IG_A + 1.0) * ls2 - IG_B / s2;
        lw[j] = lap + logprior + logtrap;
        for (int a = 0; a < D; ++a) {
            double A[D][D], e[D] = {0, 0, 0, 0}, x[D];
            memcpy(A, negH, sizeof A);
            e[a] = 1.0;
            solve4(A, e, x);                           /* x_a = C_aa */
            pc[j][a] = Phi(-(th[a] - theta0[a]) / sqrt(x[a]));
        }
    }
    double mx = -INFINITY;
    for (int j = 0; j < NODES; ++j) mx = fmax(mx, lw[j]);
    double s = 0.0;
    for (int j = 0; j < NODES; ++j) s += exp(lw[j] - mx);
    const double lse = mx + log(s);
    for (int a = 0; a < D; ++a) Sc[a] = 0.0;
    for (int j = 0; j < NODES; ++j) {
        const double pj = exp(lw[j] - lse);
        for (int a = 0; a < D; ++a) Sc[a] += pj * pc[j][a];
    }
}

/* Statistics 1 - P_a(y), a = 0..3, for a list of outcome indices ((y0 m + y1) m + y2) m + y3. */
void orc_basket_table(int n, const double *theta0, const int64_t *idx, int64_t count, double *out) {
    const int64_t m = n + 1;
    for (int64_t t = 0; t < count; ++t) {
        int64_t v = idx[t];
        int32_t y[D];
        for (int a = D - 1; a >= 0; --a) {
            y[a] = (int32_t)(v % m);
            v /= m;
        }
        orc_basket_complement(y, n, theta0, out + D * t);
    }
}

/* Tiles are (centre theta [4], configuration b): bit a of b set when H_a: theta_a <= theta_0a
 * holds on the tile.  Simulation k draws arm a, patient j from word a*n + j.  The statistic is
 * S_b = min_{a in b} (1 - P_a(y)); the design rejects a true null (the FWER event) when
 * S_b < cut (cut = 0.15 for the 85% rule).  Outputs as orc_hier4_sim. */
static double *g_bmemo = NULL;
static unsigned char *g_bhave = NULL;
static int g_bmemo_n = -1;
static double g_bmemo_t0[D];

void orc_basket_sim(int64_t n_tiles, const double *theta, const int32_t *cfg, const int32_t *sims,
                    uint64_t seed, int n, const double *theta0, double cut, int32_t *R, int64_t *sumT,
                    double *S, int64_t s_stride) {
    const int64_t m = n + 1;
    if (g_bmemo_n != n || memcmp(g_bmemo_t0, theta0, sizeof g_bmemo_t0) != 0) {
        free(g_bmemo);
        free(g_bhave);
        g_bmemo = (double *)malloc(sizeof(double) * D * m * m * m * m);
        g_bhave = (unsigned char *)calloc((size_t)(m * m * m * m), 1);
        g_bmemo_n = n;
        memcpy(g_bmemo_t0, theta0, sizeof g_bmemo_t0);
    }
    for (int64_t t = 0; t < n_tiles; ++t) {
        uint32_t T[D];
        for (int a = 0; a < D; ++a) T[a] = orc_bern_threshold(theta[t * D + a]);
        int32_t r = 0;
        int64_t st[D] = {0, 0, 0, 0};
        for (int32_t k = 0; k < sims[t]; ++k) {
            int32_t y[D];
            for (int a = 0; a < D; ++a) {
                y[a] = 0;
                for (int j = 0; j < n; ++j)
                    if (orc_word(seed, (uint32_t)k, (uint32_t)(a * n + j)) < T[a]) y[a] += 1;
            }
            const int64_t idx = ((y[0] * m + y[1]) * m + y[2]) * m + y[3];
            if (!g_bhave[idx]) {
                orc_basket_complement(y, n, theta0, g_bmemo + D * idx);
                g_bhave[idx] = 1;
            }
            const double *Sc = g_bmemo + D * idx;
            double s = INFINITY;
            for (int a = 0; a < D; ++a)
                if ((cfg[t] >> a) & 1) s = fmin(s, Sc[a]);
            if (s < cut) {
                r += 1;
                for (int a = 0; a < D; ++a) st[a] += y[a];
            }
            if (S) S[t * s_stride + k] = s;
        }
        R[t] = r;
        if (sumT)
            for (int a = 0; a < D; ++a) sumT[t * D + a] = st[a];
    }
}
