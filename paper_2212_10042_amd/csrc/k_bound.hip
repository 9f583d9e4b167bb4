// k_bound.hip -- float64 bound of each tile, eight lanes per tile.
//
//  * Clopper-Pearson upper bound Beta^{-1}(1-delta; R+1, N-R) (Section 5.1): the regularized
//    incomplete beta function by the continued fraction of DLMF 8.17.22 (modified Lentz
//    evaluation), inverted by bracketed Newton steps on log(1 - I_x).
//  * Tilewise Optimized Tilt-Bound inf_q max_{v in vertices} U(theta, v, q, a) (Theorem 1,
//    Remark 3, Theorem 3) and the calibration target sup_q min_v U^{-1}(theta, v, q, alpha)
//    (Section 6.2), exponential-family form psi(theta, v, q) = A(theta + q v) - A(theta)
//    (Example 1).  Both objectives are quasi-convex (quasi-concave) in q (Theorem 2), so a
//    parallel section search over s = log(q - 1) in [-30, 30] finds the optimum.
//  Log-partition A(theta): normal location sum theta^2/2; independent Bernoulli arms with n
//  patients each in logit parametrisation, n * sum softplus(theta_a).
#include <math.h>

#include "cse_internal.h"
#include "kernels.h"

namespace cse {

constexpr int MAXV = 64;   // vertices per tile handled by the bound kernel

__device__ __forceinline__ double softplus(double x) {
    return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x));
}

// ---- regularized incomplete beta ----
__device__ double lbeta(double a, double b) { return lgamma(a) + lgamma(b) - lgamma(a + b); }

// 1 / (1 + d1/(1 + d2/(1 + ...))) of DLMF 8.17.22 by the modified Lentz method.
__device__ double beta_cf(double a, double b, double x) {
    const double tiny = 1e-300, eps = 1e-16;
    double f = 1.0, C = 1.0, D = 0.0;
    for (int j = 1; j <= 100000; ++j) {
        double dj;
        if (j & 1) {
            const double m = (double)((j - 1) / 2);
            dj = -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0));
        } else {
            const double m = (double)(j / 2);
            dj = m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
        }
        D = 1.0 + dj * D;
        if (fabs(D) < tiny) D = tiny;
        C = 1.0 + dj / C;
        if (fabs(C) < tiny) C = tiny;
        D = 1.0 / D;
        const double delta = C * D;
        f *= delta;
        if (fabs(delta - 1.0) < eps) break;
    }
    return 1.0 / f;
}

// Upper tail Q(x) = 1 - I_x(a, b) given lb = log B(a, b): the fraction is evaluated on the
// side where it converges fast (x < (a+1)/(a+b+2) for I_x(a,b), else I_{1-x}(b,a) directly).
__device__ double ibeta_upper(double a, double b, double x, double lb) {
    if (x <= 0.0) return 1.0;
    if (x >= 1.0) return 0.0;
    const double lf = a * log(x) + b * log1p(-x) - lb;
    if (x < (a + 1.0) / (a + b + 2.0)) return 1.0 - exp(lf) / a * beta_cf(a, b, x);
    return exp(lf) / b * beta_cf(b, a, 1.0 - x);
}

// Clopper-Pearson (1 - delta) upper bound: the x with P(Binom(N, x) <= R) = Q(x; R+1, N-R) = delta.
// Start at the normal approximation mean + z sd (z = upper delta quantile of N(0,1), from the
// host), then Newton steps on log Q - log delta kept inside a bisection bracket.
__device__ double cp_upper(int R, int N, double delta, double z) {
    if (R >= N) return 1.0;
    const double a = (double)R + 1.0, b = (double)(N - R);
    const double lb = lbeta(a, b);
    const double ld = log(delta);
    double lo = 0.0, hi = 1.0;
    const double mu = a / (a + b), sd = sqrt(a * b / ((a + b) * (a + b) * (a + b + 1.0)));
    double x = mu + z * sd;
    if (!(x > 0.0 && x < 1.0)) x = 0.5 * (mu + 1.0);
    for (int it = 0; it < 200; ++it) {
        const double Q = ibeta_upper(a, b, x, lb);
        if (Q > delta)
            lo = x;
        else
            hi = x;
        const double ldens = (a - 1.0) * log(x) + (b - 1.0) * log1p(-x) - lb;
        // Newton step on h(x) = log Q(x) - log delta, h'(x) = -density / Q
        double xn = x + (log(Q) - ld) * Q / exp(ldens);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        const bool done = fabs(xn - x) <= 1e-15 * x || hi - lo <= 1e-16 * hi;
        x = xn;
        if (done) break;
    }
    return x;
}

// ---- optimisation over q ----
// GB lanes cooperate on one tile: each round they evaluate the objective at GB interior points
// of the current bracket of s = log(q - 1), keep the two intervals around the best point
// (valid for a unimodal objective, Theorem 2) and shrink the bracket by (GB+1)/2.
constexpr int GB = 8;
constexpr int SECTION_ROUNDS = 20;     // 60 * (2/9)^20 ~ 5e-12

template <int FAM>
__device__ __forceinline__ double part(int n, int d, const double *th, double q, const double *v) {
    double s = 0.0;
    for (int a = 0; a < d; ++a) {
        const double x = th[a] + q * v[a];
        s += (FAM == FAM_NORMAL) ? 0.5 * x * x : softplus(x);
    }
    return (FAM == FAM_NORMAL) ? s : (double)n * s;
}

template <int FAM, bool INV>
__device__ double objective(int n, int d, const double *th, const double *V, int nv,
                            const double *psi1, double A0, double loga, double s) {
    const double q = 1.0 + exp(s);
    double w = INV ? 1e300 : -1e300;
    for (int j = 0; j < nv; ++j) {
        const double psiq = part<FAM>(n, d, th, q, V + j * d) - A0;
        if (INV)
            w = fmin(w, q / (q - 1.0) * (loga - psiq / q + psi1[j]));
        else
            w = fmax(w, (1.0 - 1.0 / q) * loga + psiq / q - psi1[j]);
    }
    return w;
}

template <int FAM, bool INV>
__device__ double section_search(int lane, int n, int d, const double *th, const double *V, int nv,
                                 const double *psi1, double A0, double loga, double *s_best) {
    const double sg = INV ? -1.0 : 1.0;    // minimise sg * objective
    double lo = -30.0, hi = 30.0;
    double best = INFINITY, bs = 0.0;
    for (int r = 0; r < SECTION_ROUNDS; ++r) {
        const double h = (hi - lo) / (double)(GB + 1);
        double f = sg * objective<FAM, INV>(n, d, th, V, nv, psi1, A0, loga, lo + (lane + 1) * h);
        if (f != f) f = INFINITY;
        int jm = lane;
#pragma unroll
        for (int m = 1; m < GB; m <<= 1) {
            const double fo = __shfl_xor(f, m);
            const int jo = __shfl_xor(jm, m);
            if (fo < f || (fo == f && jo < jm)) {
                f = fo;
                jm = jo;
            }
        }
        if (f < best) {
            best = f;
            bs = lo + (jm + 1) * h;
        }
        const double nlo = lo + jm * h;
        hi = lo + (jm + 2) * h;
        lo = nlo;
    }
    *s_best = bs;
    return sg * best;
}

// mode 0: validate (CP then tilt), mode 1: invert (alpha', k), mode 2: tilt of given a.
template <int FAM>
__global__ __launch_bounds__(256) void k_bound(int mode, int n, int d, int64_t n_tiles,
                                               const double *__restrict__ theta,
                                               const int32_t *__restrict__ vert_off,
                                               const double *__restrict__ verts,
                                               const int32_t *__restrict__ N,
                                               const uint32_t *__restrict__ R,
                                               const double *__restrict__ a_in, double level,
                                               double zq, double *__restrict__ out,
                                               double *__restrict__ q_out,
                                               int32_t *__restrict__ k_out,
                                               double *__restrict__ cp_out) {
    __shared__ double s_psi1[256 / GB][MAXV];
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % GB, grp = threadIdx.x / GB;
    int64_t t = gid / GB;
    const bool valid = t < n_tiles;
    if (!valid) t = n_tiles - 1;   // idle groups shadow the last tile and write nothing
    double th[MAX_D];
    for (int a = 0; a < d; ++a) th[a] = theta[t * d + a];
    const double *V = verts + (int64_t)vert_off[t] * d;
    const int nv = min(vert_off[t + 1] - vert_off[t], MAXV);
    const double zero[MAX_D] = {0.0, 0.0, 0.0, 0.0};
    const double A0 = part<FAM>(n, d, th, 0.0, zero);
    for (int j = lane; j < nv; j += GB) s_psi1[grp][j] = part<FAM>(n, d, th, 1.0, V + j * d) - A0;
    __syncthreads();
    const double *psi1 = s_psi1[grp];

    if (mode == 1) {
        double sb;
        const double val = section_search<FAM, true>(lane, n, d, th, V, nv, psi1, A0, log(level), &sb);
        if (valid && lane == 0) {
            const double ap = exp(val);
            out[t] = ap;
            if (q_out) q_out[t] = 1.0 + exp(sb);
            if (k_out) k_out[t] = (int32_t)floor(((double)N[t] + 1.0) * ap);
        }
        return;
    }
    double a;
    if (mode == 0) {
        a = cp_upper((int)R[t], N[t], level, zq);
        if (valid && lane == 0 && cp_out) cp_out[t] = a;
    } else {
        a = a_in[t];
    }
    if (a <= 0.0 || a >= 1.0) {
        if (valid && lane == 0) {
            out[t] = a <= 0.0 ? 0.0 : 1.0;
            if (q_out) q_out[t] = a <= 0.0 ? INFINITY : 1.0;
        }
        return;
    }
    double sb;
    const double val = section_search<FAM, false>(lane, n, d, th, V, nv, psi1, A0, log(a), &sb);
    if (valid && lane == 0) {
        out[t] = fmin(exp(val), 1.0);
        if (q_out) q_out[t] = 1.0 + exp(sb);
    }
}

// Upper delta quantile of N(0, 1) by bisection on erfc (host; starting point of the CP Newton).
static double normal_upper_quantile(double delta) {
    double lo = -40.0, hi = 40.0;
    for (int i = 0; i < 200; ++i) {
        const double m = 0.5 * (lo + hi);
        if (0.5 * erfc(m / sqrt(2.0)) > delta)
            lo = m;
        else
            hi = m;
    }
    return 0.5 * (lo + hi);
}

hipError_t launch_bound(const Platten &P, int mode, const uint32_t *R, const double *a_in,
                        double level, double *out, double *q_out, int32_t *k_out, double *cp_out,
                        hipStream_t st) {
    const int bs = 256;
    const int64_t threads = P.n_tiles * GB;
    const int64_t grid = (threads + bs - 1) / bs;
    const double zq = mode == 0 ? normal_upper_quantile(level) : 0.0;
    if (P.family == FAM_NORMAL)
        hipLaunchKernelGGL(k_bound<FAM_NORMAL>, dim3((uint32_t)grid), dim3(bs), 0, st, mode, P.n_per_arm,
                           P.d, P.n_tiles, P.d_theta, P.d_vert_off, P.d_verts, P.d_N, R, a_in, level,
                           zq, out, q_out, k_out, cp_out);
    else
        hipLaunchKernelGGL(k_bound<FAM_BINOM>, dim3((uint32_t)grid), dim3(bs), 0, st, mode, P.n_per_arm,
                           P.d, P.n_tiles, P.d_theta, P.d_vert_off, P.d_verts, P.d_N, R, a_in, level,
                           zq, out, q_out, k_out, cp_out);
    return hipGetLastError();
}

}  // namespace cse
