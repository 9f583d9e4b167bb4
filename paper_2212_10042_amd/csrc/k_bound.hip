// k_bound.hip -- float64 bound of each tile, eight lanes per tile.
//
//  * Clopper-Pearson upper bound Beta^{-1}(1-delta; R+1, N-R) (Section 6.1): the regularized
//    incomplete beta function by the continued fraction of DLMF 8.17.22 (modified Lentz
//    evaluation), inverted by bracketed Newton steps on log(1 - I_x).
//  * Tilewise Optimized Tilt-Bound inf_q max_{v in vertices} U(theta, v, q, a) (Theorem 1,
//    Remark 3, Theorem 3) and the calibration target sup_q min_v U^{-1}(theta, v, q, alpha)
//    (Section 7.2), exponential-family form psi(theta, v, q) = A(theta + q v) - A(theta)
//    (Example 1).  Both objectives are quasi-convex (quasi-concave) in q (Theorem 2), so a
//    parallel section search over s = log(q - 1) in [-30, 30] finds the optimum.
//  Log-partition A(theta): normal location sum theta^2/2; independent Bernoulli arms with n
//  patients each in logit parametrisation, n * sum softplus(theta_a).
#include <math.h>

#include "cse_internal.h"
#include "fp64_math.hpp"
#include "kernels.h"

namespace cse {

constexpr int MAXV = 64;   // vertices per tile handled by the bound kernel

// 1/d for finite d > 0: hardware reciprocal and two Newton steps (within an ulp).
__device__ __forceinline__ double rcp_nr(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// log(1 + e^x), the Bernoulli log partition per patient in logit parametrisation:
// max(x, 0) + log1p(e), e = exp(-|x|), log1p(e) = 2 atanh(e / (2 + e)).
__device__ __forceinline__ double softplus(double x) {
    const double e = exp_cw(-fabs(x));
    return fmax(x, 0.0) + log1p_from_u(e * rcp_nr(2.0 + e));
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
// R = 0 has the closed form 1 - delta^(1/N).  Otherwise start at the normal approximation
// mean + z sd (z = upper delta quantile of N(0,1), from the host) and take Halley steps on
// h(x) = log Q(x) - log delta inside a bisection bracket:  h' = -r, h'' = -r (g + r) with
// r = density / Q and g = (a-1)/x - (b-1)/(1-x) the log-derivative of the density.
__device__ double cp_upper(int R, int N, double delta, double z) {
    if (R >= N) return 1.0;
    if (R == 0) return -expm1(log(delta) / (double)N);
    const double a = (double)R + 1.0, b = (double)(N - R);
    const double lb = lbeta(a, b);
    const double ld = log(delta);
    double lo = 0.0, hi = 1.0;
    const double mu = a / (a + b), sd = sqrt(a * b / ((a + b) * (a + b) * (a + b + 1.0)));
    double x = mu + z * sd;
    if (!(x > 0.0 && x < 1.0)) x = 0.5 * (mu + 1.0);
    for (int it = 0; it < 60; ++it) {
        const double Q = ibeta_upper(a, b, x, lb);
        if (Q > delta)
            lo = x;
        else
            hi = x;
        const double h = log(Q) - ld;
        const double r = exp((a - 1.0) * log(x) + (b - 1.0) * log1p(-x) - lb) / Q;
        const double g = (a - 1.0) / x - (b - 1.0) / (1.0 - x);
        // Newton step h / r, Halley's correction 1 / (1 + h (g + r) / (2 r)) when it is moderate
        const double newton = h / r;
        const double fac = 1.0 + 0.5 * newton * (g + r);
        double xn = x + ((fac > 0.5 && fac < 2.0) ? newton / fac : newton);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        // stop when the residual is below the rounding noise of log Q (~1e-13, from the log-beta
        // normalisation), or the bracket has collapsed
        if (fabs(h) < 4e-12 || hi - lo <= 4e-16 * hi) break;
        x = xn;
    }
    return x;
}

// ---- optimisation over q ----
// GB lanes cooperate on one tile: each round they evaluate the objective at GB interior points
// of the current bracket of s = log(q - 1), keep the two intervals around the best point
// (valid for a unimodal objective, Theorem 2) and shrink the bracket by (GB+1)/2.
constexpr int GB = 8;
// bracket 60 * (2/9)^12 ~ 9e-7 in s; near the optimum the objective is quadratic in s, so the
// best sampled value is within (1/2) f'' (9e-7)^2 of the optimum (~1e-11 for |f''| ~ 50)
constexpr int SECTION_ROUNDS = 12;
// one lane per tile from this many tiles on (measured: at 33 k and 60 k tiles the serial chain
// of evaluations per tile is slower than the cooperative search; at 2^20 tiles the single
// lane's fewer evaluations win)
constexpr int64_t BOUND_ONE_LANE_TILES = 262144;

template <int FAM, int D>
__device__ __forceinline__ double part(int n, const double *th, double q, const double *v) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double x = th[a] + q * v[a];
        s += (FAM == FAM_NORMAL) ? 0.5 * x * x : softplus(x);
    }
    return (FAM == FAM_NORMAL) ? s : (double)n * s;
}

template <int FAM>
__device__ __forceinline__ double part1(int n, double x) {
    return (FAM == FAM_NORMAL) ? 0.5 * x * x : (double)n * softplus(x);
}

// Distinct displacement values per arm that the general form shares between vertices.
constexpr int SHU = 2;

// One tile's data for the search over q (D = parameter dimension, a compile-time constant so
// the per-arm arrays stay in registers).
template <int D>
struct TileGeom {
    int n, nv;
    bool box;                 // whole box: the objective is separable over arms
    double th[D], r[D];
    double A0a[D];            // per-arm log partition at theta (box form)
    double p1[D][2];          // per-arm psi(theta, -r / +r, 1) (box form)
    const double *V;          // vertex displacements (general form)
    const double *psi1;       // per-vertex psi(theta, v, 1) (general form)
    double A0;
    // general form with shared terms: the vertices' displacement along arm a takes at most SHU
    // distinct values uv[a * SHU + .] (the pieces of a box cut at the null boundaries of the
    // grids here keep two: the box's own faces), and bit a of vidx[j] picks vertex j's value;
    // each arm's log-partition term is then evaluated once per distinct value instead of once
    // per vertex
    bool shared;
    const double *uv;
    const uint8_t *vidx;
};

// log-partition term of one arm at natural parameter x (without the patient count)
template <int FAM>
__device__ __forceinline__ double arm_term(double x) {
    return (FAM == FAM_NORMAL) ? 0.5 * x * x : softplus(x);
}

// max over the tile's vertices of  psi(theta, v, q) / q - psi(theta, v, 1).
// For a whole box A is a sum over arms and the vertices are all sign patterns (+-r_a), so the
// maximum is the sum over arms of the larger of the two one-arm terms (same value as the
// vertex loop, 2d instead of d 2^d log-partition terms).
template <int FAM, int D>
__device__ double max_tilt_term(const TileGeom<D> &T, double q) {
    const double iq = 1.0 / q;
    if (T.box) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double lo = (part1<FAM>(T.n, T.th[a] - q * T.r[a]) - T.A0a[a]) * iq - T.p1[a][0];
            const double hi = (part1<FAM>(T.n, T.th[a] + q * T.r[a]) - T.A0a[a]) * iq - T.p1[a][1];
            s += fmax(lo, hi);
        }
        return s;
    }
    double w = -1e300;
    if (T.shared) {
        double sp[D][SHU];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int c = 0; c < SHU; ++c) sp[a][c] = arm_term<FAM>(T.th[a] + q * T.uv[a * SHU + c]);
        for (int j = 0; j < T.nv; ++j) {
            const uint32_t code = T.vidx[j];
            double sum = 0.0;   // the same terms in the same order as part()
#pragma unroll
            for (int a = 0; a < D; ++a) sum += ((code >> a) & 1u) ? sp[a][1] : sp[a][0];
            const double psiq = ((FAM == FAM_NORMAL) ? sum : (double)T.n * sum) - T.A0;
            w = fmax(w, psiq * iq - T.psi1[j]);
        }
        return w;
    }
    for (int j = 0; j < T.nv; ++j) {
        const double psiq = part<FAM, D>(T.n, T.th, q, T.V + j * D) - T.A0;
        w = fmax(w, psiq * iq - T.psi1[j]);
    }
    return w;
}

// log U (forward, max over vertices) or log U^{-1} (inverse, min over vertices); the inverse's
// min over v of q/(q-1) (log alpha - psi_q/q + psi_1) is q/(q-1) (log alpha - max_v(...)).
template <int FAM, int D, bool INV>
__device__ double objective(const TileGeom<D> &T, double loga, double s) {
    const double q = 1.0 + exp_cw(s);
    const double m = max_tilt_term<FAM, D>(T, q);
    return INV ? q / (q - 1.0) * (loga - m) : (1.0 - 1.0 / q) * loga + m;
}

// A starting point for the search: expanding the log-partition differences to second order,
// psi(theta, v, q) / q - psi(theta, v, 1) ~ (q - 1) v'H v / 2 with H the Fisher information at
// theta, so log U ~ (1 - 1/q) L + (q - 1) sigma^2 / 2 (sigma^2 the largest v'H v over the
// vertices), least at q = sqrt(2 |L| / sigma^2); returns log(q - 1), or NaN when the expansion
// gives no point.  The same point serves the inverse (its optimum differs at higher order).
template <int FAM, int D>
__device__ double start_s(const TileGeom<D> &T, double L) {
    double h[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (FAM == FAM_NORMAL) {
            h[a] = 1.0;
        } else {
            const double p = 1.0 / (1.0 + exp(-T.th[a]));
            h[a] = (double)T.n * p * (1.0 - p);
        }
    }
    double s2 = 0.0;
    if (T.box) {
#pragma unroll
        for (int a = 0; a < D; ++a) s2 += T.r[a] * T.r[a] * h[a];
    } else {
        for (int j = 0; j < T.nv; ++j) {
            double t = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) t += T.V[j * D + a] * T.V[j * D + a] * h[a];
            s2 = fmax(s2, t);
        }
    }
    if (!(s2 > 0.0) || !(L < 0.0)) return NAN;
    const double q = sqrt(-2.0 * L / s2);
    return q > 1.0 + 1e-9 ? log(q - 1.0) : NAN;
}

template <int FAM, int D, bool INV>
__device__ double section_search(int lane, const TileGeom<D> &T, double loga, double *s_best) {
    const double sg = INV ? -1.0 : 1.0;    // minimise sg * objective
    double lo = -30.0, hi = 30.0;
    double best = INFINITY, bs = 0.0;
    int rounds = SECTION_ROUNDS;
    // a first round on s0 +- 1 around the expansion's optimum: when its best point is interior
    // the optimum lies in the two intervals around it (unimodal objective) and 9 more rounds
    // reach the full search's bracket width (0.44 (2/9)^9 < 60 (2/9)^12); else the full search
    const double s0 = start_s<FAM, D>(T, loga);   // the same in every lane of the tile
    if (s0 > -29.0 && s0 < 29.0) {
        const double l0 = s0 - 1.0, h = 2.0 / (double)(GB + 1);
        double f = sg * objective<FAM, D, INV>(T, loga, l0 + (lane + 1) * h);
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
        if (jm > 0 && jm < GB - 1 && f < INFINITY) {
            best = f;
            bs = l0 + (jm + 1) * h;
            lo = l0 + jm * h;
            hi = l0 + (jm + 2) * h;
            rounds = SECTION_ROUNDS - 3;
        }
    }
    for (int r = 0; r < rounds; ++r) {
        const double h = (hi - lo) / (double)(GB + 1);
        double f = sg * objective<FAM, D, INV>(T, loga, lo + (lane + 1) * h);
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

// One lane per tile: Brent's minimisation on s over the same bracket (Brent, Algorithms for
// Minimization without Derivatives, 1973): a parabola through the three best points when its
// vertex falls well inside the bracket, else a golden-section step into the larger part; stops
// when the bracket around the best point is within BRENT_TOL in s (the objective is quadratic
// near its optimum, so the best value is within ~f'' BRENT_TOL^2 of the optimum).  The
// objective is unimodal in s (Theorem 2), so the bracket keeps the optimum; the best evaluated
// point is returned, as by the cooperative search.  Fewer evaluations than a golden-section
// search to the same bracket (about 15 against 40), for launches with enough tiles to fill the
// chip with one lane per tile.
constexpr double BRENT_TOL = 2e-7;
constexpr int BRENT_MAXIT = 80;

template <int FAM, int D, bool INV>
__device__ double brent_search(const TileGeom<D> &T, double loga, double *s_best) {
    const double sg = INV ? -1.0 : 1.0;    // minimise sg * objective
    const double cg = 0.3819660112501051;  // (3 - sqrt 5) / 2
    auto ev = [&](double x) {
        const double f = sg * objective<FAM, D, INV>(T, loga, x);
        return f != f ? INFINITY : f;
    };
    double a = -30.0, b = 30.0;
    double x, w, v, fx, fw, fv;
    double d = 0.0, e = 0.0;
    // three points around the expansion's optimum s0: when the middle one is lowest the optimum
    // lies within s0 +- 1 (the objective is unimodal), else on the side of the lower end; the
    // search then starts from those points with a parabolic step.  The start changes the work,
    // not the optimum found (to BRENT_TOL).
    const double s0 = start_s<FAM, D>(T, loga);
    bool seeded = false;
    if (s0 > -29.0 && s0 < 29.0) {
        const double sl = s0 - 1.0, sh = s0 + 1.0;
        const double fl = ev(sl), fm = ev(s0), fh = ev(sh);
        if (fm < INFINITY) {
            seeded = true;
            if (fm <= fl && fm <= fh) {
                a = sl;
                b = sh;
                x = s0, fx = fm;
                w = sl, fw = fl;
                v = sh, fv = fh;
            } else if (fl < fm) {   // the optimum lies below s0
                b = s0;
                x = sl, fx = fl;
                w = s0, fw = fm;
                v = s0, fv = fm;
            } else {                // above s0
                a = s0;
                x = sh, fx = fh;
                w = s0, fw = fm;
                v = s0, fv = fm;
            }
            e = b - a;
        }
    }
    if (!seeded) {
        x = a + cg * (b - a);
        w = x;
        v = x;
        fx = ev(x);
        fw = fx;
        fv = fx;
    }
    for (int it = 0; it < BRENT_MAXIT; ++it) {
        const double xm = 0.5 * (a + b);
        const double tol1 = 0.5 * BRENT_TOL, tol2 = BRENT_TOL;
        if (fabs(x - xm) <= tol2 - 0.5 * (b - a)) break;
        bool golden = true;
        if (fabs(e) > tol1) {   // parabola through x, w, v
            const double r = (x - w) * (fx - fv);
            double q = (x - v) * (fx - fw);
            double p = (x - v) * q - (x - w) * r;
            q = 2.0 * (q - r);
            if (q > 0.0) p = -p;
            else q = -q;
            const double etemp = e;
            e = d;
            if (fabs(p) < fabs(0.5 * q * etemp) && p > q * (a - x) && p < q * (b - x)) {
                d = p / q;
                const double u = x + d;
                if (u - a < tol2 || b - u < tol2) d = xm >= x ? tol1 : -tol1;
                golden = false;
            }
        }
        if (golden) {
            e = x >= xm ? a - x : b - x;
            d = cg * e;
        }
        const double u = fabs(d) >= tol1 ? x + d : x + (d > 0.0 ? tol1 : -tol1);
        const double fu = ev(u);
        if (fu <= fx) {
            if (u >= x) a = x;
            else b = x;
            v = w;
            fv = fw;
            w = x;
            fw = fx;
            x = u;
            fx = fu;
        } else {
            if (u < x) a = u;
            else b = u;
            if (fu <= fw || w == x) {
                v = w;
                fv = fw;
                w = u;
                fw = fu;
            } else if (fu <= fv || v == x || v == w) {
                v = u;
                fv = fu;
            }
        }
    }
    *s_best = x;
    return sg * fx;
}

template <int L, int FAM, int D, bool INV>
__device__ __forceinline__ double search(int lane, const TileGeom<D> &T, double loga, double *s_best) {
    if constexpr (L == 1)
        return brent_search<FAM, D, INV>(T, loga, s_best);
    else
        return section_search<FAM, D, INV>(lane, T, loga, s_best);
}

__global__ void k_negate1(double *x) { x[0] = -x[0]; }

// mode 0: validate (CP then tilt), mode 1: invert (alpha', k), mode 2: tilt of given a,
// mode 3: lower validation bound (Remark 2: the tilt of 1 - cp_lower = cp_upper(N - R), then
// lower = 1 - that; cp_out receives cp_lower).
// L lanes per tile: GB (cooperative section search, 256-thread blocks of 32 tiles) or 1
// (Brent's search, 64-thread blocks of 64 tiles).  The per-tile vertex rows live in dynamic LDS
// sized for mv vertices (the launch's largest tile), bound_lds_bytes: sized for the 64-vertex
// maximum, one-lane blocks would hold 38 KB each and a CU would fit only one wave per SIMD.
static size_t bound_lds_bytes(int d, int tpb, int mv) {
    return (size_t)tpb * ((size_t)mv * sizeof(double) + (size_t)d * SHU * sizeof(double) + (size_t)mv);
}
template <int FAM, int D, int L>
__global__ __launch_bounds__(L == 1 ? 64 : 256) void k_bound(int mode, int n, int64_t n_tiles, int mv,
                                               const double *__restrict__ theta,
                                               const int32_t *__restrict__ vert_off,
                                               const double *__restrict__ verts,
                                               const double *__restrict__ radii,
                                               const int32_t *__restrict__ is_box,
                                               const int32_t *__restrict__ N,
                                               const uint32_t *__restrict__ R,
                                               const double *__restrict__ a_in, double level,
                                               const double *__restrict__ cp_tbl,
                                               const int64_t *__restrict__ cp_base,
                                               double *__restrict__ out,
                                               double *__restrict__ q_out,
                                               int32_t *__restrict__ k_out,
                                               double *__restrict__ cp_out) {
    constexpr int TPB = L == 1 ? 64 : 256 / GB;   // tiles per block
    static_assert(L == 1 || L == GB, "lanes per tile");
    extern __shared__ double s_dyn[];
    double *s_psi1 = s_dyn;                                          // [TPB][mv]
    double *s_uv = s_dyn + (size_t)TPB * mv;                         // [TPB][D * SHU]
    uint8_t *s_vidx = reinterpret_cast<uint8_t *>(s_uv + TPB * D * SHU);   // [TPB][mv]
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % L, grp = threadIdx.x / L;
    int64_t t = gid / L;
    const bool valid = t < n_tiles;
    if (!valid) t = n_tiles - 1;   // idle groups shadow the last tile and write nothing
    TileGeom<D> T;
    T.n = n;
    T.box = is_box[t] != 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T.th[a] = theta[t * D + a];
        T.r[a] = radii[t * D + a];
    }
    T.V = verts + (int64_t)vert_off[t] * D;
    T.nv = min(vert_off[t + 1] - vert_off[t], mv);
    double zero[D];
#pragma unroll
    for (int a = 0; a < D; ++a) zero[a] = 0.0;
    T.A0 = part<FAM, D>(n, T.th, 0.0, zero);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T.A0a[a] = part1<FAM>(n, T.th[a]);
        T.p1[a][0] = part1<FAM>(n, T.th[a] - T.r[a]) - T.A0a[a];
        T.p1[a][1] = part1<FAM>(n, T.th[a] + T.r[a]) - T.A0a[a];
    }
    T.shared = false;
    if (!T.box) {
        for (int j = lane; j < T.nv; j += L) s_psi1[grp * mv + j] = part<FAM, D>(n, T.th, 1.0, T.V + j * D) - T.A0;
        // distinct displacement values per arm, in order of first appearance (every lane of the
        // group finds the same ones); an arm with one value repeats it in the second slot
        bool shared = true;
        double v0[D], v1[D];
        bool two[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            v0[a] = T.V[a];
            v1[a] = v0[a];
            two[a] = false;
        }
        for (int j = 0; j < T.nv; ++j) {
            uint32_t code = 0u;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double x = T.V[j * D + a];
                if (x != v0[a]) {
                    if (!two[a]) {
                        v1[a] = x;
                        two[a] = true;
                    } else if (x != v1[a]) {
                        shared = false;
                    }
                    code |= 1u << a;
                }
            }
            if (j % L == lane) s_vidx[grp * mv + j] = (uint8_t)code;
        }
        if (lane == 0)
#pragma unroll
            for (int a = 0; a < D; ++a) {
                s_uv[grp * D * SHU + a * SHU] = v0[a];
                s_uv[grp * D * SHU + a * SHU + 1] = v1[a];
            }
        T.shared = shared;
    }
    __syncthreads();
    T.psi1 = s_psi1 + grp * mv;
    T.vidx = s_vidx + grp * mv;
    T.uv = s_uv + grp * D * SHU;

    if (mode == 1) {
        double sb;
        const double val = search<L, FAM, D, true>(lane, T, log(level), &sb);
        if (valid && lane == 0) {
            const double ap = exp(val);
            out[t] = ap;
            if (q_out) q_out[t] = 1.0 + exp_cw(sb);
            if (k_out) k_out[t] = (int32_t)floor(((double)N[t] + 1.0) * ap);
        }
        return;
    }
    double a;
    if (mode == 0) {
        a = cp_tbl[cp_base[t] + (int64_t)R[t]];
        if (valid && lane == 0 && cp_out) cp_out[t] = a;
    } else if (mode == 3) {
        const uint32_t r = min(R[t], (uint32_t)N[t]);
        a = cp_tbl[cp_base[t] + (int64_t)((uint32_t)N[t] - r)];
        if (valid && lane == 0 && cp_out) cp_out[t] = 1.0 - a;
    } else {
        a = a_in[t];
    }
    const bool lower = mode == 3;
    if (a <= 0.0 || a >= 1.0) {
        if (valid && lane == 0) {
            const double ub = a <= 0.0 ? 0.0 : 1.0;
            out[t] = lower ? 1.0 - ub : ub;
            if (q_out) q_out[t] = a <= 0.0 ? INFINITY : 1.0;
        }
        return;
    }
    double sb;
    const double val = search<L, FAM, D, false>(lane, T, log(a), &sb);
    if (valid && lane == 0) {
        const double ub = fmin(exp(val), 1.0);
        out[t] = lower ? 1.0 - ub : ub;
        if (q_out) q_out[t] = 1.0 + exp(sb);
    }
}


// ---- Taylor comparison bound (Section 4.3) and the gradient-guided worst vertex ----
// Per tile: h_a = sup over the box of d^2 A / d theta_a^2 (1 for the normal family; for a
// binomial arm n p (1 - p) at the point of [theta_a - r_a, theta_a + r_a] nearest 0), which
// bounds the second-order remainder of a rejection probability in the exponential family;
// the bound f + g.v + (1/2) sum_a h_a v_a^2 is convex in v, so its maximum over the tile is at
// a vertex: that vertex (first on ties) is also the tile's worst-case candidate point.
template <int FAM, int D>
__global__ void k_taylor(int n, int64_t n_tiles, const double *__restrict__ theta,
                         const double *__restrict__ radii, const int32_t *__restrict__ vert_off,
                         const double *__restrict__ verts, const double *__restrict__ f,
                         const double *__restrict__ g, double *__restrict__ bound,
                         int32_t *__restrict__ vertex, double *__restrict__ point) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    double th[D], h[D], gg[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        th[a] = theta[t * D + a];
        gg[a] = g[t * D + a];
        if (FAM == FAM_NORMAL) {
            h[a] = 1.0;
        } else {
            const double r = radii[t * D + a], lo = th[a] - r, hi = th[a] + r;
            const double x = (lo <= 0.0 && hi >= 0.0) ? 0.0 : (hi < 0.0 ? hi : lo);
            const double p = 1.0 / (1.0 + exp(-x));
            h[a] = (double)n * p * (1.0 - p);
        }
    }
    const int32_t v0 = vert_off[t], nv = vert_off[t + 1] - v0;
    double best = -INFINITY;
    int jb = 0;
    for (int j = 0; j < nv; ++j) {
        double val = f[t];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double v = verts[(int64_t)(v0 + j) * D + a];
            val += gg[a] * v + 0.5 * h[a] * v * v;
        }
        if (val > best) {
            best = val;
            jb = j;
        }
    }
    bound[t] = fmin(best, 1.0);
    if (vertex) vertex[t] = jb;
    if (point)
#pragma unroll
        for (int a = 0; a < D; ++a) point[t * D + a] = th[a] + verts[(int64_t)(v0 + jb) * D + a];
}

hipError_t launch_taylor(const Platten &P, const double *f, const double *g, double *bound, int32_t *vertex,
                         double *point, hipStream_t st) {
    const dim3 grid((uint32_t)((P.n_tiles + 255) / 256));
#define CSE_TAYLOR_LAUNCH(FAM, D)                                                                         \
    hipLaunchKernelGGL((k_taylor<FAM, D>), grid, dim3(256), 0, st, P.n_per_arm, P.n_tiles, P.d_theta, P.d_radii, \
                       P.d_vert_off, P.d_verts, f, g, bound, vertex, point)
    if (P.family == FAM_NORMAL && P.d == 1)
        CSE_TAYLOR_LAUNCH(FAM_NORMAL, 1);
    else if (P.family == FAM_BINOM && P.d == 2)
        CSE_TAYLOR_LAUNCH(FAM_BINOM, 2);
    else if (P.family == FAM_BINOM && P.d == 4)
        CSE_TAYLOR_LAUNCH(FAM_BINOM, 4);
    else
        return hipErrorInvalidValue;
#undef CSE_TAYLOR_LAUNCH
    return hipGetLastError();
}

// ---- confidence sets from calibration (Section 8) ----
// Per tile: kept when its test does not reject the observed statistic, s_i >= lambda_i
// (compared in the precision of the design's keys: float64 outcome statistics for the 2-arm
// design, float32 otherwise), and the range of e(theta) = c0 + sum_a c_a g(theta_a) over the
// tile: g = identity, min / max over the vertices (exact on a polytope); g = expit, the sum of
// each term's extremes over the tile's bounding box (exact on a box, enclosing on a clipped
// tile).  Tiles not kept get the empty range (+inf, -inf).
struct ConfCoef {
    double c[4];
    double c0;
};

template <int D>
__global__ void k_confset(int64_t n_tiles, const double *__restrict__ theta, const int32_t *__restrict__ vert_off,
                          const double *__restrict__ verts, const double *__restrict__ s_obs, int64_t s_stride,
                          const double *__restrict__ lam, ConfCoef cf, int link, bool f64_keys,
                          int32_t *__restrict__ keep, double *__restrict__ e_lo, double *__restrict__ e_hi,
                          double *__restrict__ e_min, double *__restrict__ e_max) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const double s = s_obs[t * s_stride], L = lam[t];
    const bool kp = f64_keys ? !(s < L) : !((float)s < (float)L);
    double th[D], mn[D], mx[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        th[a] = theta[t * D + a];
        mn[a] = INFINITY;
        mx[a] = -INFINITY;
    }
    const int32_t v0 = vert_off[t], nv = vert_off[t + 1] - v0;
    double lo = INFINITY, hi = -INFINITY;
    for (int j = 0; j < nv; ++j) {
        double val = cf.c0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double x = th[a] + verts[(int64_t)(v0 + j) * D + a];
            val += cf.c[a] * x;
            mn[a] = fmin(mn[a], x);
            mx[a] = fmax(mx[a], x);
        }
        lo = fmin(lo, val);
        hi = fmax(hi, val);
    }
    if (link == 1) {
        lo = hi = cf.c0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double u = cf.c[a] / (1.0 + exp(-mn[a])), w = cf.c[a] / (1.0 + exp(-mx[a]));
            lo += fmin(u, w);
            hi += fmax(u, w);
        }
    }
    keep[t] = kp ? 1 : 0;
    e_lo[t] = lo;
    e_hi[t] = hi;
    e_min[t] = kp ? lo : INFINITY;
    e_max[t] = kp ? -hi : INFINITY;   // negated: both reductions take a minimum
}

hipError_t launch_confset(const Platten &P, const double *s_obs, int64_t s_stride, const double *lam,
                          const double *coef, int link, int32_t *keep, double *e_lo, double *e_hi,
                          double *e_range, hipStream_t st) {
    ConfCoef cf{};
    for (int a = 0; a < P.d; ++a) cf.c[a] = coef[a];
    cf.c0 = coef[P.d];
    const dim3 grid((uint32_t)((P.n_tiles + 255) / 256));
    const bool f64 = P.design.kind == CSE_BINOM2_Z;
    // the per-tile minima land in two float64 workspaces of n_tiles entries
    double *wmin = P.d_apw, *wmax = P.d_lamw;
#define CSE_CONF_LAUNCH(D)                                                                                    \
    hipLaunchKernelGGL((k_confset<D>), grid, dim3(256), 0, st, P.n_tiles, P.d_theta, P.d_vert_off, P.d_verts,   \
                       s_obs, s_stride, lam, cf, link, f64, keep, e_lo, e_hi, wmin, wmax)
    if (P.n_tiles == 0)
        ;   // nothing kept: the reductions below give the empty range (+inf, -inf)
    else if (P.d == 1)
        CSE_CONF_LAUNCH(1);
    else if (P.d == 2)
        CSE_CONF_LAUNCH(2);
    else if (P.d == 4)
        CSE_CONF_LAUNCH(4);
    else
        return hipErrorInvalidValue;
#undef CSE_CONF_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_min(P, wmin, nullptr, P.n_tiles, e_range, st)) != hipSuccess) return e;
    if ((e = launch_min(P, wmax, nullptr, P.n_tiles, e_range + 1, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_negate1, dim3(1), dim3(1), 0, st, e_range + 1);
    return hipGetLastError();
}

// Clopper-Pearson once per (N class, R) present in this call: mark, then solve marked entries.
// flip: mark N - R instead (the lower bound, cp_lower(R) = 1 - cp_upper(N - R)).
__global__ void k_cp_mark(int64_t n_tiles, const uint32_t *__restrict__ R, const int32_t *__restrict__ N,
                          const int64_t *__restrict__ cp_base, bool flip, uint32_t *__restrict__ mark) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t r = min(R[t], (uint32_t)N[t]);
    mark[cp_base[t] + (flip ? (uint32_t)N[t] - r : r)] = 1u;
}

__global__ void k_cp_table(const int32_t *__restrict__ cls_N, const int64_t *__restrict__ cls_off,
                           const uint32_t *__restrict__ mark, double delta, double zq,
                           double *__restrict__ tbl) {
    const int c = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = cls_N[c];
    if (r > n) return;
    const int64_t e = cls_off[c] + r;
    if (mark[e]) tbl[e] = cp_upper(r, n, delta, zq);
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
    if (mode == 0 || mode == 3) {
        hipError_t e = launch_zero(P.d_cp_mark, (size_t)P.n_cp * sizeof(uint32_t), st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_cp_mark, dim3((uint32_t)((P.n_tiles + 255) / 256)), dim3(256), 0, st,
                           P.n_tiles, R, P.d_N, P.d_cp_base, mode == 3, P.d_cp_mark);
        const double zq = normal_upper_quantile(level);
        hipLaunchKernelGGL(k_cp_table, dim3((uint32_t)((P.max_cls_N + 1 + 63) / 64), (uint32_t)P.n_cls),
                           dim3(64), 0, st, P.d_cls_N, P.d_cls_off, P.d_cp_mark, level, zq, P.d_cp_tbl);
    }
    // enough tiles to give every SIMD work with one lane per tile: Brent's search (fewer
    // evaluations); otherwise GB lanes per tile shorten each tile's chain of evaluations
    const bool one_lane = P.n_tiles >= BOUND_ONE_LANE_TILES;
    const int bs = one_lane ? 64 : 256;
    const int64_t threads = P.n_tiles * (one_lane ? 1 : GB);
    const int64_t grid = (threads + bs - 1) / bs;
    const int mv = std::min(std::max(P.max_nv, 1), MAXV);
#define CSE_BOUND_LAUNCH(FAM, D)                                                                        \
    do {                                                                                                \
        if (one_lane)                                                                                   \
            hipLaunchKernelGGL((k_bound<FAM, D, 1>), dim3((uint32_t)grid), dim3(bs),                     \
                               bound_lds_bytes(D, 64, mv), st,      mode, P.n_per_arm,                  \
                               P.n_tiles, mv, P.d_theta, P.d_vert_off, P.d_verts, P.d_radii, P.d_is_box, P.d_N, R, \
                               a_in, level, P.d_cp_tbl, P.d_cp_base, out, q_out, k_out, cp_out);          \
        else                                                                                            \
            hipLaunchKernelGGL((k_bound<FAM, D, GB>), dim3((uint32_t)grid), dim3(bs),                   \
                               bound_lds_bytes(D, 256 / GB, mv), st,      mode, P.n_per_arm,            \
                               P.n_tiles, mv, P.d_theta, P.d_vert_off, P.d_verts, P.d_radii, P.d_is_box, P.d_N, R, \
                               a_in, level, P.d_cp_tbl, P.d_cp_base, out, q_out, k_out, cp_out);          \
    } while (0)
    if (P.family == FAM_NORMAL && P.d == 1)
        CSE_BOUND_LAUNCH(FAM_NORMAL, 1);
    else if (P.family == FAM_BINOM && P.d == 2)
        CSE_BOUND_LAUNCH(FAM_BINOM, 2);
    else if (P.family == FAM_BINOM && P.d == 4)
        CSE_BOUND_LAUNCH(FAM_BINOM, 4);
    else
        return hipErrorInvalidValue;
#undef CSE_BOUND_LAUNCH
    return hipGetLastError();
}

}  // namespace cse
