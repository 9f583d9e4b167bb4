// k_bound.hip -- float64 bound of each tile, one thread per tile.
//
//  * Clopper-Pearson upper bound Beta^{-1}(1-delta; R+1, N-R) (Section 5.1): the regularized
//    incomplete beta function by the continued fraction of DLMF 8.17.22 (modified Lentz
//    evaluation), inverted by bracketed Newton steps on log(1 - I_x).
//  * Tilewise Optimized Tilt-Bound inf_q max_{v in vertices} U(theta, v, q, a) (Theorem 1,
//    Remark 3, Theorem 3) and the calibration target sup_q min_v U^{-1}(theta, v, q, alpha)
//    (Section 6.2), exponential-family form psi(theta, v, q) = A(theta + q v) - A(theta)
//    (Example 1).  Both objectives are quasi-convex (quasi-concave) in q (Theorem 2), so a
//    golden-section search over s = log(q - 1) in [-30, 30] finds the optimum.
#include <math.h>

#include "cse_internal.h"
#include "kernels.h"

namespace cse {

constexpr int MAXV = 64;   // vertices per tile handled by the bound kernel

__device__ __forceinline__ double softplus(double x) {
    return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x));
}

// Log-partition A(theta): normal location sum theta^2/2; independent Bernoulli arms with
// n patients each in logit parametrisation, n * sum softplus(theta_a).
__device__ double log_partition(int fam, int n, int d, const double *th, double q, const double *v) {
    double s = 0.0;
    for (int a = 0; a < d; ++a) {
        const double x = th[a] + q * v[a];
        s += (fam == FAM_NORMAL) ? 0.5 * x * x : softplus(x);
    }
    return (fam == FAM_NORMAL) ? s : (double)n * s;
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

// x^a (1-x)^b / (a B(a,b)) * fraction  =  I_x(a,b)   where the fraction converges fast.
__device__ double ibeta_front(double a, double b, double x) {
    return exp(a * log(x) + b * log1p(-x) - lbeta(a, b)) / a * beta_cf(a, b, x);
}

// Upper tail Q(x) = 1 - I_x(a, b), accurate when it is small.
__device__ double ibeta_upper(double a, double b, double x) {
    if (x <= 0.0) return 1.0;
    if (x >= 1.0) return 0.0;
    if (x < (a + 1.0) / (a + b + 2.0)) return 1.0 - ibeta_front(a, b, x);
    return ibeta_front(b, a, 1.0 - x);
}

// Clopper-Pearson (1 - delta) upper bound: the x with P(Binom(N, x) <= R) = Q(x; R+1, N-R) = delta.
__device__ double cp_upper(int R, int N, double delta) {
    if (R >= N) return 1.0;
    const double a = (double)R + 1.0, b = (double)(N - R);
    const double ld = log(delta);
    double lo = 0.0, hi = 1.0;
    double x = a / (a + b);
    for (int it = 0; it < 200; ++it) {
        const double Q = ibeta_upper(a, b, x);
        if (Q > delta)
            lo = x;
        else
            hi = x;
        const double ldens = (a - 1.0) * log(x) + (b - 1.0) * log1p(-x) - lbeta(a, b);
        // Newton step on h(x) = log Q(x) - log delta, h'(x) = -density / Q
        double xn = x + (log(Q) - ld) * Q / exp(ldens);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-15 * x || hi - lo <= 1e-16 * hi) {
            x = xn;
            break;
        }
        x = xn;
    }
    return x;
}

// ---- golden-section search over s = log(q - 1) ----
struct TileView {
    int fam, n, d, nv;
    const double *th;
    const double *V;
    double A0;
    double psi1[MAXV];
};

__device__ double obj_tilt(const TileView &T, double s, double loga) {
    const double q = 1.0 + exp(s);
    double w = -1e300;
    for (int j = 0; j < T.nv; ++j) {
        const double psiq = log_partition(T.fam, T.n, T.d, T.th, q, T.V + j * T.d) - T.A0;
        const double lu = (1.0 - 1.0 / q) * loga + psiq / q - T.psi1[j];
        w = fmax(w, lu);
    }
    return w;
}

__device__ double obj_inv(const TileView &T, double s, double loga) {
    const double q = 1.0 + exp(s);
    double w = 1e300;
    for (int j = 0; j < T.nv; ++j) {
        const double psiq = log_partition(T.fam, T.n, T.d, T.th, q, T.V + j * T.d) - T.A0;
        const double li = q / (q - 1.0) * (loga - psiq / q + T.psi1[j]);
        w = fmin(w, li);
    }
    return w;
}

// Minimise sgn * obj over s; returns s* and writes obj(s*).
template <bool INV>
__device__ double golden(const TileView &T, double loga, double *val) {
    const double g = 0.61803398874989484820;
    const double sg = INV ? -1.0 : 1.0;
    double lo = -30.0, hi = 30.0;
    double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
    double f1 = sg * (INV ? obj_inv(T, x1, loga) : obj_tilt(T, x1, loga));
    double f2 = sg * (INV ? obj_inv(T, x2, loga) : obj_tilt(T, x2, loga));
    for (int it = 0; it < 100; ++it) {
        if (f1 <= f2) {
            hi = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi - g * (hi - lo);
            f1 = sg * (INV ? obj_inv(T, x1, loga) : obj_tilt(T, x1, loga));
        } else {
            lo = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo + g * (hi - lo);
            f2 = sg * (INV ? obj_inv(T, x2, loga) : obj_tilt(T, x2, loga));
        }
    }
    const double s = 0.5 * (lo + hi);
    *val = INV ? obj_inv(T, s, loga) : obj_tilt(T, s, loga);
    return s;
}

// mode 0: validate (CP then tilt), mode 1: invert (alpha', k), mode 2: tilt of given a.
__global__ __launch_bounds__(64) void k_bound(int mode, int fam, int n, int d, int64_t n_tiles,
                                              const double *__restrict__ theta,
                                              const int32_t *__restrict__ vert_off,
                                              const double *__restrict__ verts,
                                              const int32_t *__restrict__ N,
                                              const uint32_t *__restrict__ R,
                                              const double *__restrict__ a_in, double level,
                                              double *__restrict__ out, double *__restrict__ q_out,
                                              int32_t *__restrict__ k_out,
                                              double *__restrict__ cp_out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    TileView T;
    T.fam = fam;
    T.n = n;
    T.d = d;
    T.th = theta + t * d;
    T.V = verts + (int64_t)vert_off[t] * d;
    T.nv = min(vert_off[t + 1] - vert_off[t], MAXV);
    const double zero[MAX_D] = {0.0, 0.0, 0.0, 0.0};
    T.A0 = log_partition(fam, n, d, T.th, 0.0, zero);
    for (int j = 0; j < T.nv; ++j) T.psi1[j] = log_partition(fam, n, d, T.th, 1.0, T.V + j * d) - T.A0;

    if (mode == 1) {
        double val;
        const double s = golden<true>(T, log(level), &val);
        const double ap = exp(val);
        out[t] = ap;
        if (q_out) q_out[t] = 1.0 + exp(s);
        if (k_out) k_out[t] = (int32_t)floor(((double)N[t] + 1.0) * ap);
        return;
    }
    double a;
    if (mode == 0) {
        a = cp_upper((int)R[t], N[t], level);
        if (cp_out) cp_out[t] = a;
    } else {
        a = a_in[t];
    }
    if (a <= 0.0) {
        out[t] = 0.0;
        if (q_out) q_out[t] = INFINITY;
        return;
    }
    if (a >= 1.0) {
        out[t] = 1.0;
        if (q_out) q_out[t] = 1.0;
        return;
    }
    double val;
    const double s = golden<false>(T, log(a), &val);
    out[t] = fmin(exp(val), 1.0);
    if (q_out) q_out[t] = 1.0 + exp(s);
}

hipError_t launch_bound(const Platten &P, int mode, const uint32_t *R, const double *a_in,
                        double level, double *out, double *q_out, int32_t *k_out, double *cp_out,
                        hipStream_t st) {
    const int bs = 64;
    const int64_t grid = (P.n_tiles + bs - 1) / bs;
    hipLaunchKernelGGL(k_bound, dim3((uint32_t)grid), dim3(bs), 0, st, mode, P.family, P.n_per_arm,
                       P.d, P.n_tiles, P.d_theta, P.d_vert_off, P.d_verts, P.d_N, R, a_in, level,
                       out, q_out, k_out, cp_out);
    return hipGetLastError();
}

}  // namespace cse
