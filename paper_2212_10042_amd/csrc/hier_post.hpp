// hier_post.hpp -- float64 posterior of the four-arm hierarchical model of the basket case
// study (Section 10.1), per thread, for counts y_a out of n_a patients on arm a (arm 0 control):
//   theta_a | mu, s2 ~ N(mu, s2), mu ~ N(-1.34, 100), s2 ~ InvGamma(0.0005, 0.000005).
//
//   * mu is integrated out: theta | s2 ~ N(m0 1, Sigma), Sigma = s2 I + 100 11^T, with precision
//     Q = (I - c 11^T) / s2, c = 100 / (s2 + 400) (Sherman-Morrison);
//   * per node s2_j (90 nodes equally spaced in log s2 on [log 1e-6, log 1e3]) the conditional
//     posterior of theta is replaced by its Laplace approximation: the mode by Newton's method on
//     sum_a [y_a theta_a - n_a softplus(theta_a)] - (theta - m0)^T Q (theta - m0) / 2, whose
//     negative Hessian D - beta 11^T (D_a = n_a p_a (1 - p_a) + 1/s2, beta = c / s2) makes every
//     step, determinant and covariance C = D^{-1} + g u u^T (u = D^{-1} 1,
//     g = beta / (1 - beta sum u)) cost O(arms);
//   * node log weight: Laplace evidence l(mode) + log|Q|/2 - log|D - beta 11^T|/2, plus the log
//     inverse-gamma density of s2_j and the log trapezoid weight in log s2 (ds2 = s2 dlog s2),
//     normalised by a running log-sum-exp in float64;
//   * P_i = sum_j pi_j Phi(z_ij), z_ij = (mode_i - mode_0) / sqrt(C_ii + C_00 - 2 C_i0); the
//     complements 1 - P_i are summed directly as sum_j pi_j Phi(-z_ij) (relative precision where
//     P_i is near 1);
//   * with FULL, the node mixture's moments: means and variances of theta_a and of
//     theta_i - theta_0 (variance = mean over nodes of C + spread of the modes, accumulated
//     about a fixed reference point so that no large terms cancel).
#pragma once
#include <math.h>

#include "cse_internal.h"
#include "fp64_math.hpp"

namespace cse {

constexpr int HP_NODES = 90;
// Newton stops after applying a step below this size: convergence is quadratic near the mode,
// so the remaining error is of the order of its square (~1e-12), below the 1e-10 step a fully
// converged iteration would still take.
constexpr double HP_NEWTON_TOL = 1e-6;

// Per-node constants (HierNode, cse_internal.h) are computed once on the host.

// 1/d for finite d > 0: hardware reciprocal and two Newton steps (error below one ulp).
__device__ __forceinline__ double rcp_nr(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// 1/sqrt(d) for finite d > 0: hardware estimate and two Newton steps (error about one ulp).
__device__ __forceinline__ double rsq_nr(double d) {
    double y = __builtin_amdgcn_rsq(d);
    const double h = 0.5 * d;
    y = fma(y, fma(-h * y, y, 0.5), y);
    return fma(y, fma(-h * y, y, 0.5), y);
}

// expit(x), and with it softplus(x) = max(x, 0) + log1p(exp(-|x|)) from the same exponential.
__device__ __forceinline__ double hp_expit(double x) {
    const double e = exp_cw(-fabs(x));          // in (0, 1]
    const double r = rcp_nr(1.0 + e);           // argument in (1, 2]
    return x >= 0.0 ? r : 1.0 - r;
}
__device__ __forceinline__ double hp_expit_softplus(double x, double &sp) {
    const double e = exp_cw(-fabs(x));
    const double r = rcp_nr(1.0 + e);
    sp = fmax(x, 0.0) + log1p_unit(e);
    return x >= 0.0 ? r : 1.0 - r;
}

// 1 / x_a for four finite positive x_a with one reciprocal: the reciprocal of their product
// times the other three factors (a few ulp; the products stay far inside the double range for
// the values here: 1 + e in (1, 2], curvatures in [1e-3, 1e6 + n/4]).  The treatment arms'
// cofactors are x0 times the product of the other two in ascending arm order, so arms 1..3
// with equal x get bit-identical results and ties between them stay exact ties.
__device__ __forceinline__ void rcp4(const double x[4], double r[4]) {
    const double x12 = x[1] * x[2], x13 = x[1] * x[3], x23 = x[2] * x[3];
    const double inv = rcp_nr(x[0] * (x12 * x[3]));
    r[0] = inv * (x12 * x[3]);
    r[1] = inv * (x[0] * x23);
    r[2] = inv * (x[0] * x13);
    r[3] = inv * (x[0] * x12);
}

struct HierSummary {
    double P[3];      // P(theta_i > theta_0 | data), i = 1..3
    double Sc[3];     // 1 - P_i
    double mean[4];   // mixture mean of theta_a                    (FULL only)
    double var[4];    // mixture variance of theta_a                (FULL only)
    double dvar[3];   // mixture variance of theta_i - theta_0      (FULL only)
};

// Posterior of counts y[4] out of n[4].  WARM starts each node's Newton iterations at the
// previous node's mode (the converged mode is the same; only the path differs).  Bit i-1 of
// `need` asks for P_i and 1 - P_i (the others are left 0).
template <bool FULL, bool WARM>
__device__ __forceinline__ void hier_posterior(const int y[4], const double n[4], const HierNode *__restrict__ nodes,
                                               HierSummary &out, int *newton_steps = nullptr, int need = 7) {
    const double M0 = -1.34;
    // empirical logits: the first Newton start and the fixed reference point of the moment
    // sums (any fixed point serves; held in float32 to keep registers for the trial state)
    float th0[4];
    double th[4];
    for (int a = 0; a < 4; ++a) {
        th[a] = log((y[a] + 0.5) / (n[a] - y[a] + 0.5));
        th0[a] = (float)th[a];
    }
    float thp[4] = {th0[0], th0[1], th0[2], th0[3]};   // WARM: the mode two nodes back (float32)

    double wmax = -INFINITY, wsum = 0.0;
    double accP[3] = {0.0, 0.0, 0.0}, accS[3] = {0.0, 0.0, 0.0};
    double m1[4] = {0.0, 0.0, 0.0, 0.0}, m2[4] = {0.0, 0.0, 0.0, 0.0}, d2[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < HP_NODES; ++j) {
        const HierNode nd = nodes[j];   // uniform across lanes
        const double inv_s2 = nd.inv_s2, c = nd.c, beta = nd.beta;
        if (!WARM)
            for (int a = 0; a < 4; ++a) th[a] = th0[a];
        if (WARM)   // the modes move smoothly in log s2: start from the line through the last two
            for (int a = 0; a < 4; ++a) {
                const double cur = th[a];
                if (j >= 2) th[a] = 2.0 * cur - (double)thp[a];
                thp[a] = (float)cur;
            }
        double D[4], u[4], gam = 0.0;
        for (int it = 0; it < 100; ++it) {
            double dsum = 0.0;
            for (int a = 0; a < 4; ++a) dsum += th[a] - M0;
            double g[4], su = 0.0, q1[4], r1[4];
            for (int a = 0; a < 4; ++a) q1[a] = 1.0 + exp_cw(-fabs(th[a]));
            rcp4(q1, r1);   // expit(|theta_a|)
            for (int a = 0; a < 4; ++a) {
                const double p = th[a] >= 0.0 ? r1[a] : 1.0 - r1[a];
                // Q (theta - m0) = ((theta_a - m0) - c sum_b (theta_b - m0)) / s2
                g[a] = (double)y[a] - n[a] * p - ((th[a] - M0) - c * dsum) * inv_s2;
                D[a] = n[a] * p * (1.0 - p) + inv_s2;
            }
            rcp4(D, u);
            for (int a = 0; a < 4; ++a) su += u[a];
            gam = beta * rcp_nr(1.0 - beta * su);
            double ug = 0.0;
            for (int a = 0; a < 4; ++a) ug += u[a] * g[a];
            double mx = 0.0;
            for (int a = 0; a < 4; ++a) {
                const double step = u[a] * g[a] + gam * u[a] * ug;   // (D - beta 11^T)^{-1} g
                th[a] += step;
                mx = fmax(mx, fabs(step));
            }
            if (newton_steps) *newton_steps += 1;
            if (mx < HP_NEWTON_TOL) break;
        }
        // curvature at the final mode; log|D| as the log of the product (each D_a lies in
        // [1e-3, 1e6 + n/4], so the product of four cannot overflow)
        double su = 0.0, prodD = 1.0, ll = 0.0, dsum = 0.0, sq = 0.0;
        {
            double ex[4], q1[4], r1[4], q2[4], r2[4];
            for (int a = 0; a < 4; ++a) {
                ex[a] = exp_cw(-fabs(th[a]));
                q1[a] = 1.0 + ex[a];
                q2[a] = 2.0 + ex[a];   // in (2, 3]
            }
            rcp4(q1, r1);   // expit(|theta_a|)
            rcp4(q2, r2);   // for softplus: log1p(e) = 2 atanh(e / (2 + e))
            for (int a = 0; a < 4; ++a) {
                const double p = th[a] >= 0.0 ? r1[a] : 1.0 - r1[a];
                const double sp = fmax(th[a], 0.0) + log1p_from_u(ex[a] * r2[a]);
                D[a] = n[a] * p * (1.0 - p) + inv_s2;
                prodD *= D[a];
                ll += y[a] * th[a] - n[a] * sp;
                const double e = th[a] - M0;
                dsum += e;
                sq += e * e;
            }
        }
        rcp4(D, u);
        for (int a = 0; a < 4; ++a) su += u[a];
        gam = beta * rcp_nr(1.0 - beta * su);
        const double logdet_negH = log(prodD * (1.0 - beta * su));   // both factors in range
        const double quad = (sq - c * dsum * dsum) * inv_s2;
        const double lw = ll - 0.5 * quad - 0.5 * logdet_negH + nd.lconst;
        double pc[3], pr[3], vd[3];
        for (int i = 1; i < 4; ++i) {
            const double du = u[i] - u[0];
            vd[i - 1] = u[i] + u[0] + gam * du * du;
            pc[i - 1] = 0.0;
            pr[i - 1] = 0.0;
            if ((need >> (i - 1)) & 1) {
                const double zs = (th[i] - th[0]) * rsq_nr(2.0 * vd[i - 1]);
                if (FULL) {   // one tail gives both: the smaller side directly, the other as 1 - it
                    const double tail = 0.5 * erfc(fabs(zs));
                    pc[i - 1] = zs >= 0.0 ? tail : 1.0 - tail;   // Phi(-z)
                    pr[i - 1] = zs >= 0.0 ? 1.0 - tail : tail;   // Phi(z)
                } else {
                    pc[i - 1] = 0.5 * erfc(zs);
                }
            }
        }
        if (lw > wmax) {
            const double sc = exp(wmax - lw);   // 0 on the first node
            wsum *= sc;
            for (int i = 0; i < 3; ++i) accS[i] *= sc;
            if (FULL) {
                for (int i = 0; i < 3; ++i) {
                    accP[i] *= sc;
                    d2[i] *= sc;
                }
                for (int a = 0; a < 4; ++a) {
                    m1[a] *= sc;
                    m2[a] *= sc;
                }
            }
            wmax = lw;
        }
        const double wj = exp(lw - wmax);
        wsum += wj;
        for (int i = 0; i < 3; ++i) accS[i] += wj * pc[i];
        if (FULL) {
            for (int i = 0; i < 3; ++i) {
                accP[i] += wj * pr[i];
                const double e = (th[i + 1] - th[0]) - (th0[i + 1] - th0[0]);
                d2[i] += wj * (vd[i] + e * e);
            }
            for (int a = 0; a < 4; ++a) {
                const double e = th[a] - th0[a];
                m1[a] += wj * e;
                m2[a] += wj * (u[a] + gam * u[a] * u[a] + e * e);   // C_aa + (mode - ref)^2
            }
        }
    }
    for (int i = 0; i < 3; ++i) out.Sc[i] = accS[i] / wsum;
    if (FULL) {
        for (int i = 0; i < 3; ++i) out.P[i] = accP[i] / wsum;
        double em[4];
        for (int a = 0; a < 4; ++a) {
            em[a] = m1[a] / wsum;                       // mean - reference
            out.mean[a] = th0[a] + em[a];
            out.var[a] = m2[a] / wsum - em[a] * em[a];
        }
        for (int i = 0; i < 3; ++i) {
            const double ed = em[i + 1] - em[0];
            out.dvar[i] = d2[i] / wsum - ed * ed;
        }
    }
}

// Basket design (Section 10.1's validation case study): arm a against its fixed rate,
// theta0[a] = logit p_0a; the hierarchical model is on the offsets theta_a - theta0[a], so in
// theta the prior mean is m0 + theta0[a] per arm with the same covariance, and the statistic
// of arm a is P(theta_a > theta0[a] | y).  Writes the complements
// Sc[a] = sum_j pi_j Phi(-(mode_a - theta0[a]) / sqrt(C_aa)), C_aa = u_a + g u_a^2.
__device__ __forceinline__ void basket_posterior(const int y[4], double n, const double theta0[4],
                                                 const HierNode *__restrict__ nodes, double Sc[4]) {
    const double M0 = -1.34;
    double mean[4], th[4];
    for (int a = 0; a < 4; ++a) {
        mean[a] = M0 + theta0[a];
        th[a] = log((y[a] + 0.5) / (n - y[a] + 0.5));
    }
    double wmax = -INFINITY, wsum = 0.0, acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < HP_NODES; ++j) {
        const HierNode nd = nodes[j];   // uniform across lanes
        const double inv_s2 = nd.inv_s2, c = nd.c, beta = nd.beta;
        double D[4], u[4], gam = 0.0;
        for (int it = 0; it < 100; ++it) {   // warm start: the previous node's mode
            double dsum = 0.0;
            for (int a = 0; a < 4; ++a) dsum += th[a] - mean[a];
            double g[4], su = 0.0;
            for (int a = 0; a < 4; ++a) {
                const double p = hp_expit(th[a]);
                g[a] = (double)y[a] - n * p - ((th[a] - mean[a]) - c * dsum) * inv_s2;
                D[a] = n * p * (1.0 - p) + inv_s2;
                u[a] = rcp_nr(D[a]);
                su += u[a];
            }
            gam = beta * rcp_nr(1.0 - beta * su);
            double ug = 0.0;
            for (int a = 0; a < 4; ++a) ug += u[a] * g[a];
            double mx = 0.0;
            for (int a = 0; a < 4; ++a) {
                const double step = u[a] * g[a] + gam * u[a] * ug;
                th[a] += step;
                mx = fmax(mx, fabs(step));
            }
            if (mx < HP_NEWTON_TOL) break;
        }
        double su = 0.0, prodD = 1.0, ll = 0.0, dsum = 0.0, sq = 0.0;
        for (int a = 0; a < 4; ++a) {
            double sp;
            const double p = hp_expit_softplus(th[a], sp);
            D[a] = n * p * (1.0 - p) + inv_s2;
            u[a] = rcp_nr(D[a]);
            su += u[a];
            prodD *= D[a];
            ll += y[a] * th[a] - n * sp;
            const double e = th[a] - mean[a];
            dsum += e;
            sq += e * e;
        }
        gam = beta * rcp_nr(1.0 - beta * su);
        const double logdet_negH = log(prodD * (1.0 - beta * su));   // both factors in range
        const double quad = (sq - c * dsum * dsum) * inv_s2;
        const double lw = ll - 0.5 * quad - 0.5 * logdet_negH + nd.lconst;
        double pc[4];
        for (int a = 0; a < 4; ++a) {
            const double caa = u[a] + gam * u[a] * u[a];
            pc[a] = 0.5 * erfc((th[a] - theta0[a]) / sqrt(2.0 * caa));   // Phi(-z)
        }
        if (lw > wmax) {
            const double sc = exp(wmax - lw);   // 0 on the first node
            wsum *= sc;
            for (int a = 0; a < 4; ++a) acc[a] *= sc;
            wmax = lw;
        }
        const double wj = exp(lw - wmax);
        wsum += wj;
        for (int a = 0; a < 4; ++a) acc[a] += wj * pc[a];
    }
    for (int a = 0; a < 4; ++a) Sc[a] = acc[a] / wsum;
}

}  // namespace cse
