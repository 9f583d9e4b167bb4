// platten.cpp -- host side of the platten (Section 5, Definition 1): the null partition of
// each box, the vertices of every tile (float64), the Bernoulli thresholds, the design
// tables and the tile batches ("blocks") the kernels run.  Everything is uploaded once.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <chrono>
#include <tuple>

#include "cse_internal.h"
#include "kernels.h"

namespace cse {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
const char *get_error() { return g_err.c_str(); }

namespace {

// Bernoulli(expit theta) from one uniform 32-bit word u: success iff u < T,
// T = round(2^32 / (1 + exp(-theta))), clamped to [0, 2^32 - 1].
uint32_t bern_threshold(double theta) {
    double p = 1.0 / (1.0 + exp(-theta));
    double t = floor(p * 4294967296.0 + 0.5);
    if (t < 0.0) t = 0.0;
    if (t > 4294967295.0) t = 4294967295.0;
    return (uint32_t)t;
}

// Pooled two-proportion z for y0 (control) and y1 (treatment) successes out of n each;
// 0 when the pooled rate is 0 or 1.
double pooled_z(int y0, int y1, int n) {
    double pbar = (double)(y0 + y1) / (2.0 * n);
    if (pbar <= 0.0 || pbar >= 1.0) return 0.0;
    double se = sqrt(pbar * (1.0 - pbar) * 2.0 / n);
    return ((double)y1 / n - (double)y0 / n) / se;
}

// Half-space g . x <= h.
struct HalfSpace {
    double g[MAX_D];
    double h;
};

// Solve the d x d system A x = b by Gaussian elimination with partial pivoting.
bool solve(int d, double A[MAX_D][MAX_D], double b[MAX_D], double x[MAX_D]) {
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int r = c + 1; r < d; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (fabs(A[piv][c]) < 1e-12) return false;
        if (piv != c) {
            for (int j = 0; j < d; ++j) std::swap(A[c][j], A[piv][j]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < d; ++r) {
            double f = A[r][c] / A[c][c];
            for (int j = c; j < d; ++j) A[r][j] -= f * A[c][j];
            b[r] -= f * b[c];
        }
    }
    for (int r = d - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < d; ++j) s -= A[r][j] * x[j];
        x[r] = s / A[r][r];
    }
    return true;
}

// Vertices of the polytope {x : g_i . x <= h_i} (bounded by construction: it lies in a box).
// Every vertex is the solution of d active constraints; enumerate all d-subsets.
std::vector<std::vector<double>> enumerate_vertices(int d, const std::vector<HalfSpace> &H) {
    std::vector<std::vector<double>> V;
    const int m = (int)H.size();
    std::vector<int> idx(d);
    std::function<void(int, int)> rec = [&](int start, int depth) {
        if (depth == d) {
            double A[MAX_D][MAX_D], b[MAX_D], x[MAX_D];
            for (int r = 0; r < d; ++r) {
                for (int j = 0; j < d; ++j) A[r][j] = H[idx[r]].g[j];
                b[r] = H[idx[r]].h;
            }
            if (!solve(d, A, b, x)) return;
            for (int i = 0; i < m; ++i) {
                double s = 0.0;
                for (int j = 0; j < d; ++j) s += H[i].g[j] * x[j];
                if (s > H[i].h + 1e-12 * (1.0 + fabs(H[i].h))) return;
            }
            for (auto &v : V) {
                double dm = 0.0;
                for (int j = 0; j < d; ++j) dm = std::max(dm, fabs(v[j] - x[j]));
                if (dm <= 1e-12) return;
            }
            V.emplace_back(x, x + d);
            return;
        }
        for (int i = start; i < m; ++i) {
            idx[depth] = i;
            rec(i + 1, depth + 1);
        }
    };
    rec(0, 0);
    return V;
}

// 16-point Gauss-Hermite rule (weight e^{-x^2}): the nodes are the zeros of H_16, found by
// Newton's method on the orthonormal Hermite functions h_k (h_0 = pi^{-1/4},
// h_{k+1} = x sqrt(2/(k+1)) h_k - sqrt(k/(k+1)) h_{k-1}, h_16' = sqrt(32) h_15) from starting
// points bracketed by sign changes on a grid; weight 1 / (16 h_15(x)^2).
void gauss_hermite16(double *x, double *w) {
    const int n = 16;
    auto eval = [&](double t, double &hn, double &hn1) {
        double a = pow(M_PI, -0.25), b = sqrt(2.0) * t * a;
        for (int k = 1; k < n; ++k) {
            const double c = t * sqrt(2.0 / (k + 1)) * b - sqrt((double)k / (k + 1)) * a;
            a = b;
            b = c;
        }
        hn = b;
        hn1 = a;
    };
    int found = 0;
    double prev = -7.0, fp, dummy;
    eval(prev, fp, dummy);
    for (int g = 1; g <= 1400 && found < n; ++g) {
        const double t = -7.0 + 0.01 * g;
        double ft;
        eval(t, ft, dummy);
        if ((fp < 0.0) != (ft < 0.0)) {
            double r = 0.5 * (prev + t);
            for (int it = 0; it < 50; ++it) {
                double hn, hn1;
                eval(r, hn, hn1);
                const double step = hn / (sqrt(2.0 * n) * hn1);
                r -= step;
                if (fabs(step) < 1e-16 * (1.0 + fabs(r))) break;
            }
            double hn, hn1;
            eval(r, hn, hn1);
            x[found] = r;
            w[found] = 1.0 / (n * hn1 * hn1);
            ++found;
        }
        prev = t;
        fp = ft;
    }
}

// Node constants of the hierarchical posterior (Section 10.1 model: mu ~ N(-1.34, 100) integrated
// out, s2 ~ InvGamma(0.0005, 0.000005), trapezoid rule in log s2 with ds2 = s2 dlog s2).
std::vector<HierNode> hier_nodes() {
    const double TAU2 = 100.0, IG_A = 0.0005, IG_B = 0.000005;
    const double LS2_LO = log(1e-6), LS2_HI = log(1e3);
    const double h = (LS2_HI - LS2_LO) / (HIER_NODES - 1);
    std::vector<HierNode> v(HIER_NODES);
    for (int j = 0; j < HIER_NODES; ++j) {
        HierNode &nd = v[j];
        nd.ls2 = LS2_LO + h * j;
        nd.s2 = exp(nd.ls2);
        nd.inv_s2 = 1.0 / nd.s2;
        nd.c = TAU2 / (nd.s2 + 4.0 * TAU2);
        nd.beta = nd.c * nd.inv_s2;
        const double logdetQ = -(3.0 * nd.ls2 + log(nd.s2 + 4.0 * TAU2));   // determinant lemma
        const double logprior = IG_A * log(IG_B) - lgamma(IG_A) - (IG_A + 1.0) * nd.ls2 - IG_B * nd.inv_s2;
        const double logtrap = log((j == 0 || j == HIER_NODES - 1) ? 0.5 * h : h) + nd.ls2;
        nd.lconst = 0.5 * logdetQ + logprior + logtrap;
    }
    return v;
}

// Phi^{-1}(0.95) by Newton's method on Phi(z) = erfc(-z / sqrt 2) / 2.
double normal_q95() {
    double z = 1.6;
    for (int it = 0; it < 50; ++it) {
        const double f = 0.5 * erfc(-z / sqrt(2.0)) - 0.95;
        const double dens = exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
        const double step = f / dens;
        z -= step;
        if (fabs(step) < 1e-16) break;
    }
    return z;
}

// Side streams of destroyed plattens, per device, for reuse (creating one costs ~35 us and
// destroying it ~30 us; a platten is destroyed only after the device has been synchronised,
// so a cached stream is idle).  Default priority, non-blocking.
std::mutex g_stream_mu;
std::map<int, std::vector<hipStream_t>> g_stream_cache;
constexpr size_t STREAM_CACHE_MAX = 16;

hipError_t take_side_stream(int device, hipStream_t *s) {
    {
        std::lock_guard<std::mutex> g(g_stream_mu);
        auto &v = g_stream_cache[device];
        if (!v.empty()) {
            *s = v.back();
            v.pop_back();
            return hipSuccess;
        }
    }
    return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}

void give_side_stream(int device, hipStream_t s) {
    {
        std::lock_guard<std::mutex> g(g_stream_mu);
        auto &v = g_stream_cache[device];
        if (v.size() < STREAM_CACHE_MAX) {
            v.push_back(s);
            return;
        }
    }
    (void)hipStreamDestroy(s);
}

// Uploads gathered into one host buffer and copied with a single transfer into a device arena
// (one synchronous copy per arena instead of one per array: each costs ~15 us of fixed
// overhead).  The destinations are assigned when the arena is flushed and must not be read
// before; they are freed with the arena.
struct Stager {
    std::vector<unsigned char> host;
    std::vector<std::pair<void **, size_t>> dst;   // destination pointer, byte offset
    template <class T>
    void add(T **d, const T *src, size_t n) {
        *d = nullptr;
        if (n == 0) return;
        const size_t off = (host.size() + 255) & ~(size_t)255;
        host.resize(off + n * sizeof(T));
        memcpy(host.data() + off, src, n * sizeof(T));
        dst.emplace_back((void **)d, off);
    }
    int flush(Platten *P) {
        if (dst.empty()) return CSE_OK;
        void *a = nullptr;
        CSE_HIP_TRY(hipMalloc(&a, host.size()));
        P->arenas.emplace_back(a, host.size());
        CSE_HIP_TRY(hipMemcpy(a, host.data(), host.size(), hipMemcpyHostToDevice));
        for (auto &d : dst) *d.first = (unsigned char *)a + d.second;
        host.clear();
        dst.clear();
        return CSE_OK;
    }
};

template <class T>
int upload(T **dst, const T *src, size_t n) {
    if (n == 0) {
        *dst = nullptr;
        return CSE_OK;
    }
    CSE_HIP_TRY(hipMalloc((void **)dst, n * sizeof(T)));
    CSE_HIP_TRY(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice));
    return CSE_OK;
}

}  // namespace

int build_platten(const cse_design *design, int64_t n_boxes, const double *theta,
                  const double *radii, const int32_t *sims, int32_t flags, Platten *P) {
    Stager stage;   // read-only arrays: one transfer at the end of the tile setup
    if (!design || !theta || !radii || !sims || n_boxes < 1) {
        set_error("cse_platten_create: NULL argument or n_boxes < 1");
        return CSE_EINVAL;
    }
    if (design->reserved != 0) {
        set_error("cse_platten_create: design.reserved must be 0");
        return CSE_EINVAL;
    }
    const int kind = design->kind;
    int d = 0, p = 0;
    if (kind == CSE_ZTEST1) {
        d = 1;
        p = 1;
        P->family = FAM_NORMAL;
    } else if (kind == CSE_BINOM2_Z) {
        d = 2;
        p = 1;
        P->family = FAM_BINOM;
    } else if (kind == CSE_HIER4 || kind == CSE_PHASE23) {
        d = 4;
        p = 3;
        P->family = FAM_BINOM;
    } else if (kind == CSE_BASKET4) {
        d = 4;
        p = 4;
        P->family = FAM_BINOM;
        for (int a = 0; a < 4; ++a)
            if (!(fabs(design->theta0[a]) < 1e6)) {
                set_error("cse_platten_create: design.theta0 must be finite for the basket design");
                return CSE_EINVAL;
            }
    } else {
        set_error("cse_platten_create: unknown design kind");
        return CSE_EINVAL;
    }
    if (design->n_arms != d) {
        set_error("cse_platten_create: design.n_arms does not match the design kind");
        return CSE_EINVAL;
    }
    if (kind == CSE_PHASE23 && design->n_per_arm != P23_NMAX_ARM) {
        set_error("cse_platten_create: the Phase II/III design embeds n_per_arm = 350 patients per arm");
        return CSE_EUNSUPPORTED;
    }
    if (kind != CSE_PHASE23 && P->family == FAM_BINOM && design->n_per_arm != NP35) {
        set_error("cse_platten_create: binomial designs are built for n_per_arm = 35");
        return CSE_EUNSUPPORTED;
    }
    if (!(fabs(design->cut) < 1e300)) {
        set_error("cse_platten_create: design.cut must be finite");
        return CSE_EINVAL;
    }
    const bool keep_all = (flags & CSE_PLATTEN_KEEP_ALL) != 0;
    if (flags & ~CSE_PLATTEN_KEEP_ALL) {
        set_error("cse_platten_create: unknown flag");
        return CSE_EINVAL;
    }
    if (keep_all && p != 1) {
        set_error("cse_platten_create: KEEP_ALL is defined for single-hypothesis designs");
        return CSE_EINVAL;
    }
    for (int64_t i = 0; i < n_boxes; ++i) {
        if (sims[i] < 1 || sims[i] > (1 << 24)) {
            set_error("cse_platten_create: sims must lie in [1, 2^24]");
            return CSE_EINVAL;
        }
        for (int j = 0; j < d; ++j) {
            if (!(radii[i * d + j] > 0.0) || !(fabs(theta[i * d + j]) < 1e6)) {
                set_error("cse_platten_create: radii must be > 0 and theta finite");
                return CSE_EINVAL;
            }
        }
    }
    P->design = *design;
    P->d = d;
    P->p = p;
    P->n_per_arm = design->n_per_arm;
    P->n_boxes = n_boxes;
    CSE_HIP_TRY(hipGetDevice(&P->device));

    // Null hypotheses as half-spaces g . theta <= 0: z-test theta <= 0; multi-arm designs
    // (arm 0 control) theta_i - theta_0 <= 0.
    std::vector<HalfSpace> hyp(p);
    for (int j = 0; j < p; ++j) {
        HalfSpace hs{};
        if (kind == CSE_ZTEST1) {
            hs.g[0] = 1.0;
        } else {
            hs.g[j + 1] = 1.0;
            hs.g[0] = -1.0;
        }
        hs.h = 0.0;
        hyp[j] = hs;
    }

    // ---- the null partition of every box (Section 5) ----
    const int ncorner = 1 << d;
    std::vector<double> centre;   // simulation point of each tile
    if (kind == CSE_BASKET4) {
        // axis-aligned null boundaries theta_a = theta0[a]: each box is cut at the boundaries it
        // straddles and each piece with b != 0 (bit a: the piece lies in theta_a <= theta0[a])
        // is a box-shaped tile simulated at its own centre; a box's pieces by b ascending
        const double *t0 = design->theta0;
        for (int64_t i = 0; i < n_boxes; ++i) {
            const double *c = theta + i * d;
            const double *r = radii + i * d;
            double pc[4][2], pr[4][2];
            int pn[4], pin[4][2];
            for (int a = 0; a < 4; ++a) {
                const double lo = c[a] - r[a], hi = c[a] + r[a];
                if (lo < t0[a] && t0[a] < hi) {
                    pn[a] = 2;
                    pc[a][0] = 0.5 * (lo + t0[a]);
                    pr[a][0] = 0.5 * (t0[a] - lo);
                    pin[a][0] = 1;
                    pc[a][1] = 0.5 * (t0[a] + hi);
                    pr[a][1] = 0.5 * (hi - t0[a]);
                    pin[a][1] = 0;
                } else {
                    pn[a] = 1;
                    pc[a][0] = c[a];
                    pr[a][0] = r[a];
                    pin[a][0] = hi <= t0[a] ? 1 : 0;
                }
            }
            struct Piece {
                int b;
                double c[4], r[4];
            };
            std::vector<Piece> pieces;
            for (int i0 = 0; i0 < pn[0]; ++i0)
                for (int i1 = 0; i1 < pn[1]; ++i1)
                    for (int i2 = 0; i2 < pn[2]; ++i2)
                        for (int i3 = 0; i3 < pn[3]; ++i3) {
                            const int ix[4] = {i0, i1, i2, i3};
                            Piece q{};
                            for (int a = 0; a < 4; ++a) {
                                q.c[a] = pc[a][ix[a]];
                                q.r[a] = pr[a][ix[a]];
                                q.b |= pin[a][ix[a]] << a;
                            }
                            if (q.b) pieces.push_back(q);
                        }
            std::sort(pieces.begin(), pieces.end(), [](const Piece &x, const Piece &y) { return x.b < y.b; });
            for (auto &q : pieces) {
                P->tile_box.push_back(i);
                P->tile_cfg.push_back(q.b);
                P->tile_in_null.push_back(1);
                P->tile_is_box.push_back(1);
                for (int a = 0; a < d; ++a) {
                    P->tile_radii.push_back(q.r[a]);
                    centre.push_back(q.c[a]);
                }
                P->tile_nv.push_back(ncorner);
                P->vert_off.push_back((int32_t)(P->verts.size() / d));
                for (int m = 0; m < ncorner; ++m)
                    for (int a = 0; a < d; ++a) {
                        const double v = q.c[a] + (((m >> a) & 1) ? q.r[a] : -q.r[a]);
                        P->verts.push_back(v - q.c[a]);
                    }
            }
        }
    }
    for (int64_t i = 0; i < (kind == CSE_BASKET4 ? 0 : n_boxes); ++i) {
        const double *c = theta + i * d;
        const double *r = radii + i * d;
        std::vector<std::vector<double>> corners(ncorner, std::vector<double>(d));
        for (int m = 0; m < ncorner; ++m)
            for (int j = 0; j < d; ++j) corners[m][j] = c[j] + (((m >> j) & 1) ? r[j] : -r[j]);
        bool met = false;
        for (int b = 1; b < (1 << p); ++b) {
            std::vector<HalfSpace> cons;
            for (int j = 0; j < p; ++j) {
                HalfSpace hs = hyp[j];
                if (!((b >> j) & 1)) {  // complement of H_j, closed: g . x >= h
                    for (int a = 0; a < d; ++a) hs.g[a] = -hs.g[a];
                    hs.h = -hs.h;
                }
                cons.push_back(hs);
            }
            bool empty = false, inside = true;
            for (auto &hs : cons) {
                double mn = 1e300, mx = -1e300;
                for (auto &x : corners) {
                    double s = -hs.h;
                    for (int a = 0; a < d; ++a) s += hs.g[a] * x[a];
                    mn = std::min(mn, s);
                    mx = std::max(mx, s);
                }
                if (mn >= 0.0) empty = true;   // the constraint holds at most on a face
                if (mx > 0.0) inside = false;
            }
            if (empty) continue;
            std::vector<std::vector<double>> V;
            if (inside) {
                V = corners;
            } else {
                std::vector<HalfSpace> all;
                for (int a = 0; a < d; ++a) {
                    HalfSpace up{}, dn{};
                    up.g[a] = 1.0;
                    up.h = c[a] + r[a];
                    dn.g[a] = -1.0;
                    dn.h = -(c[a] - r[a]);
                    all.push_back(up);
                    all.push_back(dn);
                }
                for (auto &hs : cons) all.push_back(hs);
                V = enumerate_vertices(d, all);
                if ((int)V.size() < d + 1) continue;
                // full dimension <=> the vertex centroid satisfies every constraint strictly
                std::vector<double> cen(d, 0.0);
                for (auto &v : V)
                    for (int a = 0; a < d; ++a) cen[a] += v[a] / (double)V.size();
                bool interior = true;
                for (auto &hs : all) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) s += hs.g[a] * cen[a];
                    if (!(s < hs.h - 1e-12)) interior = false;
                }
                if (!interior) continue;
            }
            met = true;
            P->tile_box.push_back(i);
            P->tile_cfg.push_back(b);
            P->tile_in_null.push_back(1);
            P->tile_is_box.push_back(inside ? 1 : 0);
            for (int a = 0; a < d; ++a) P->tile_radii.push_back(r[a]);
            P->tile_nv.push_back((int32_t)V.size());
            P->vert_off.push_back((int32_t)(P->verts.size() / d));
            for (auto &v : V)
                for (int a = 0; a < d; ++a) P->verts.push_back(v[a] - c[a]);
        }
        if (!met && keep_all) {
            P->tile_box.push_back(i);
            P->tile_cfg.push_back(1);
            P->tile_in_null.push_back(0);
            P->tile_is_box.push_back(1);
            for (int a = 0; a < d; ++a) P->tile_radii.push_back(r[a]);
            P->tile_nv.push_back(ncorner);
            P->vert_off.push_back((int32_t)(P->verts.size() / d));
            for (auto &v : corners)
                for (int a = 0; a < d; ++a) P->verts.push_back(v[a] - c[a]);
        }
    }
    P->n_tiles = (int64_t)P->tile_box.size();
    if (P->n_tiles == 0) {
        set_error("cse_platten_create: no box meets the null hypothesis space");
        return CSE_EINVAL;
    }
    P->vert_off.push_back((int32_t)(P->verts.size() / d));
    P->tile_theta.resize(P->n_tiles * d);
    P->tile_N.resize(P->n_tiles);
    std::vector<int64_t> key_off(P->n_tiles, -1), key_stride(P->n_tiles, 64);
    for (int64_t t = 0; t < P->n_tiles; ++t) {
        for (int a = 0; a < d; ++a)
            P->tile_theta[t * d + a] = kind == CSE_BASKET4 ? centre[t * d + a] : theta[P->tile_box[t] * d + a];
        P->tile_N[t] = sims[P->tile_box[t]];
        P->max_N = std::max(P->max_N, P->tile_N[t]);
        P->total_sims += P->tile_N[t];
        if (P->tile_nv[t] > 64) {
            set_error("cse_platten_create: a tile has more than 64 vertices");
            return CSE_EUNSUPPORTED;
        }
        P->max_nv = std::max(P->max_nv, P->tile_nv[t]);
    }
    if (P->family == FAM_BINOM) {
        P->tile_T.resize(P->n_tiles * d);
        for (int64_t t = 0; t < P->n_tiles * d; ++t) P->tile_T[t] = bern_threshold(P->tile_theta[t]);
    }

    // ---- tile batches ----
    std::vector<int64_t> &blk_sims = P->blk_sims;   // n_sims per block, for the work items
    if (kind == CSE_ZTEST1) {
        std::map<int32_t, std::vector<int64_t>> byN;
        for (int64_t t = 0; t < P->n_tiles; ++t) byN[P->tile_N[t]].push_back(t);
        std::vector<Blk1> blks;
        for (auto &kv : byN) {
            auto &ts = kv.second;
            for (size_t s = 0; s < ts.size(); s += B1T) {
                Blk1 B{};
                for (int j = 0; j < B1T; ++j) {
                    B.tile[j] = -1;
                    B.theta[j] = 0.0f;
                }
                for (size_t j = 0; j < B1T && s + j < ts.size(); ++j) {
                    B.tile[j] = (int32_t)ts[s + j];
                    B.theta[j] = (float)P->tile_theta[ts[s + j]];
                }
                B.n_sims = kv.first;
                blks.push_back(B);
            }
        }
        P->n_blocks = (int64_t)blks.size();
        for (auto &B : blks) {
            blk_sims.push_back(B.n_sims);
            B.key_base = P->n_keys;
            for (int j = 0; j < B1T; ++j)
                if (B.tile[j] >= 0) key_off[B.tile[j]] = B.key_base + (int64_t)j * B.n_sims;
            P->n_keys += (int64_t)B1T * B.n_sims;
        }
        if (int e = upload((Blk1 **)&P->d_blocks, blks.data(), blks.size())) return e;
    } else if (kind == CSE_HIER4 || kind == CSE_BASKET4) {
        // distinct values per arm -> coordinates; 4 x 4 x 2 x 2 coordinate blocks per N class
        const int BD[4] = {B4N0, B4N1, B4N2, B4N3};
        std::vector<double> uv[4];
        for (int64_t t = 0; t < P->n_tiles; ++t)
            for (int a = 0; a < 4; ++a) uv[a].push_back(P->tile_theta[t * 4 + a]);
        for (int a = 0; a < 4; ++a) {
            std::sort(uv[a].begin(), uv[a].end());
            uv[a].erase(std::unique(uv[a].begin(), uv[a].end()), uv[a].end());
        }
        typedef std::tuple<int32_t, int64_t, int64_t, int64_t, int64_t> Key4;
        std::map<Key4, std::vector<Blk4>> blkmap;
        for (int64_t t = 0; t < P->n_tiles;) {
            // the tiles of one simulation point are consecutive (a box's pieces, or one basket piece)
            int64_t t1 = t;
            uint32_t bm = 0;
            while (t1 < P->n_tiles && P->tile_box[t1] == P->tile_box[t] &&
                   (kind != CSE_BASKET4 || t1 == t))
                bm |= 1u << P->tile_cfg[t1++];
            int64_t c[4];
            for (int a = 0; a < 4; ++a)
                c[a] = std::lower_bound(uv[a].begin(), uv[a].end(), P->tile_theta[t * 4 + a]) - uv[a].begin();
            Key4 key = std::make_tuple(P->tile_N[t], c[0] / BD[0], c[1] / BD[1], c[2] / BD[2], c[3] / BD[3]);
            const int slot = (int)((((c[0] % BD[0]) * BD[1] + c[1] % BD[1]) * BD[2] + c[2] % BD[2]) * BD[3] + c[3] % BD[3]);
            auto &vec = blkmap[key];
            Blk4 *B = nullptr;
            for (auto &b : vec)
                if (b.row0[slot] < 0) {
                    B = &b;
                    break;
                }
            if (!B) {
                Blk4 nb{};
                for (int j = 0; j < B4S; ++j) {
                    nb.row0[j] = -1;
                    nb.tile0[j] = -1;
                    nb.bmask[j] = 0;
                }
                uint32_t *T[4] = {nb.T0, nb.T1, nb.T2, nb.T3};
                for (int a = 0; a < 4; ++a) {
                    const int64_t base = (c[a] / BD[a]) * BD[a];
                    for (int u = 0; u < BD[a]; ++u)
                        T[a][u] = (base + u < (int64_t)uv[a].size()) ? bern_threshold(uv[a][base + u]) : 0u;
                }
                nb.n_sims = P->tile_N[t];
                vec.push_back(nb);
                B = &vec.back();
            }
            B->row0[slot] = 0;   // rows assigned below
            B->tile0[slot] = (int32_t)t;
            B->bmask[slot] = bm;
            t = t1;
        }
        std::vector<Blk4> blks;
        for (auto &kv : blkmap)
            for (auto &b : kv.second) blks.push_back(b);
        P->n_blocks = (int64_t)blks.size();
        for (auto &B : blks) {
            blk_sims.push_back(B.n_sims);
            int32_t rows = 0;
            for (int j = 0; j < B4S; ++j) {
                if (B.row0[j] < 0) continue;
                B.row0[j] = rows;
                rows += __builtin_popcount(B.bmask[j]);
            }
            B.n_rows = rows;
            P->h4_max_rows = std::max(P->h4_max_rows, rows);
            B.key_base = P->n_keys;
            for (int j = 0; j < B4S; ++j) {
                if (B.row0[j] < 0) continue;
                const int nt = __builtin_popcount(B.bmask[j]);
                for (int q = 0; q < nt; ++q) {
                    const int64_t tile = B.tile0[j] + q;
                    key_off[tile] = B.key_base + (int64_t)(B.row0[j] + q) * 64;
                    key_stride[tile] = (int64_t)rows * 64;
                }
            }
            P->n_keys += ((int64_t)B.n_sims + 63) / 64 * rows * 64;
        }
        if (int e = upload((Blk4 **)&P->d_blocks, blks.data(), blks.size())) return e;

        // posterior table of the design (once per platten)
        const std::vector<HierNode> nodes = hier_nodes();
        if (int e = upload(&P->d_hnodes, nodes.data(), nodes.size())) return e;
        const int64_t m = P->n_per_arm + 1;
        P->h4_outcomes = m * m * m * m;
        CSE_HIP_TRY(hipMalloc((void **)&P->d_h4tbl, (size_t)P->h4_outcomes * sizeof(float4)));
        const auto t0 = std::chrono::steady_clock::now();
        if (kind == CSE_BASKET4)
            CSE_HIP_TRY(launch_basket_table(P->n_per_arm, design->theta0, P->d_h4tbl, P->d_hnodes, nullptr));
        else
            CSE_HIP_TRY(launch_hier4_table(P->n_per_arm, P->d_h4tbl, P->d_hnodes, nullptr));
        CSE_HIP_TRY(hipMalloc((void **)&P->d_h4mask, (size_t)P->h4_outcomes));
        CSE_HIP_TRY(launch_h4_mask(P->d_h4tbl, P->h4_outcomes, (float)design->cut, kind == CSE_BASKET4 ? 4 : 3,
                                   P->d_h4mask, nullptr));
        CSE_HIP_TRY(hipDeviceSynchronize());
        P->table_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (kind == CSE_HIER4) {   // bracketed calibration keys: the exact path regenerates a tile's keys
            if (int e = upload(&P->d_tileT, P->tile_T.data(), P->tile_T.size())) return e;
            if (int e = upload(&P->d_cfg, P->tile_cfg.data(), P->tile_cfg.size())) return e;
            const size_t nt = (size_t)std::max<int64_t>(P->n_tiles, 1);
            CSE_HIP_TRY(hipMalloc((void **)&P->d_h4brk, nt * sizeof(float2)));
            CSE_HIP_TRY(hipMalloc((void **)&P->d_h4below, nt * sizeof(uint32_t)));
            CSE_HIP_TRY(hipMalloc((void **)&P->d_h4fb, (nt + 1) * sizeof(uint32_t)));
            CSE_HIP_TRY(hipMemset(P->d_h4fb, 0, sizeof(uint32_t)));
        }
    } else if (kind == CSE_PHASE23) {
        // one trial per lane: keys contiguous per tile, work items of p23_chunk simulations
        for (int64_t t = 0; t < P->n_tiles; ++t) {
            key_off[t] = P->n_keys;
            key_stride[t] = 64;   // contiguous: chunk c of 64 keys starts at 64 c
            P->n_keys += P->tile_N[t];
        }
        if (int e = plan_queue_items(P, P->p23_chunk, -1)) return e;
        if (int e = upload(&P->d_tileT, P->tile_T.data(), P->tile_T.size())) return e;
        if (int e = upload(&P->d_cfg, P->tile_cfg.data(), P->tile_cfg.size())) return e;
        CSE_HIP_TRY(hipMalloc((void **)&P->d_queue, sizeof(uint32_t)));
        CSE_HIP_TRY(hipMalloc((void **)&P->d_p23stats, 4 * sizeof(unsigned long long)));
        P23Args &A = P->p23;
        A.counter = P->d_queue;
        A.tileT = P->d_tileT;
        A.cfg = P->d_cfg;
        A.cut = (float)design->cut;
        double gh[32];
        gauss_hermite16(gh, gh + 16);
        if (int e = upload(&P->d_gh, gh, 32)) return e;
        A.gh = P->d_gh;
        const std::vector<HierNode> nodes = hier_nodes();
        if (int e = upload(&P->d_hnodes, nodes.data(), nodes.size())) return e;
        A.nodes = P->d_hnodes;
        A.sqrt_pi = sqrt(M_PI);
        A.z95 = normal_q95();
        // decisions of the first look (50 patients per arm) for every outcome, once per platten
        CSE_HIP_TRY(hipMalloc((void **)&P->d_p23look1, (size_t)51 * 51 * 51 * 51));
        A.look1 = P->d_p23look1;
        {
            const auto t0 = std::chrono::steady_clock::now();
            CSE_HIP_TRY(launch_p23_look1(*P, nullptr));
            CSE_HIP_TRY(hipDeviceSynchronize());
            P->table_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
    } else {
        // distinct arm values -> integer coordinates; 8 x 8 coordinate blocks per N class
        std::vector<double> u0, u1;
        for (int64_t t = 0; t < P->n_tiles; ++t) {
            u0.push_back(P->tile_theta[t * 2 + 0]);
            u1.push_back(P->tile_theta[t * 2 + 1]);
        }
        std::sort(u0.begin(), u0.end());
        u0.erase(std::unique(u0.begin(), u0.end()), u0.end());
        std::sort(u1.begin(), u1.end());
        u1.erase(std::unique(u1.begin(), u1.end()), u1.end());
        std::map<std::tuple<int32_t, int64_t, int64_t>, std::vector<Blk2>> blkmap;
        for (int64_t t = 0; t < P->n_tiles; ++t) {
            int64_t c0 = std::lower_bound(u0.begin(), u0.end(), P->tile_theta[t * 2]) - u0.begin();
            int64_t c1 = std::lower_bound(u1.begin(), u1.end(), P->tile_theta[t * 2 + 1]) - u1.begin();
            auto key = std::make_tuple(P->tile_N[t], c0 / B2U, c1 / B2V);
            auto &vec = blkmap[key];
            int slot = (int)(c0 % B2U) * B2V + (int)(c1 % B2V);
            Blk2 *B = nullptr;
            for (auto &b : vec)
                if (b.tile[slot] < 0) {
                    B = &b;
                    break;
                }
            if (!B) {
                Blk2 nb{};
                for (int j = 0; j < B2U * B2V; ++j) nb.tile[j] = -1;
                int64_t b0 = (c0 / B2U) * B2U, b1 = (c1 / B2V) * B2V;
                for (int u = 0; u < B2U; ++u)
                    nb.T0[u] = (b0 + u < (int64_t)u0.size()) ? bern_threshold(u0[b0 + u]) : 0u;
                for (int v = 0; v < B2V; ++v)
                    nb.T1[v] = (b1 + v < (int64_t)u1.size()) ? bern_threshold(u1[b1 + v]) : 0u;
                nb.n_sims = P->tile_N[t];
                vec.push_back(nb);
                B = &vec.back();
            }
            B->tile[slot] = (int32_t)t;
        }
        std::vector<Blk2> blks;
        for (auto &kv : blkmap)
            for (auto &b : kv.second) {
                blks.push_back(b);
                P->blk_row.push_back(std::get<1>(kv.first));
                P->blk_col.push_back(std::get<2>(kv.first));
            }
        P->n_blocks = (int64_t)blks.size();
        for (auto &B : blks) {
            blk_sims.push_back(B.n_sims);
            // one 16-byte record per simulation of the block (chunks of 64, the last one padded)
            B.key_base = P->n_keys;
            for (int j = 0; j < B2U * B2V; ++j)
                if (B.tile[j] >= 0) {
                    key_off[B.tile[j]] = B.key_base;   // the block's first record
                    key_stride[B.tile[j]] = j;         // the tile's slot u * 8 + v
                }
            P->n_keys += ((int64_t)B.n_sims + 63) / 64 * 64;
        }
        stage.add((Blk2 **)&P->d_blocks, blks.data(), blks.size());

        // design tables of the pooled z test
        const int n = P->n_per_arm, n1 = n + 1;
        P->n_outcomes = n1 * n1;
        std::vector<int32_t> cut(n1);
        std::vector<double> S(n1 * n1);
        for (int y0 = 0; y0 <= n; ++y0) {
            cut[y0] = n1;   // no y1 rejects
            for (int y1 = 0; y1 <= n; ++y1) {
                double z = pooled_z(y0, y1, n);
                S[y0 * n1 + y1] = -z;
                if (z > design->cut && cut[y0] == n1) cut[y0] = y1;
            }
            // the kernels use {y1 >= c(y0)}: this needs z increasing in y1 for fixed y0
            for (int y1 = 0; y1 <= n; ++y1)
                if ((pooled_z(y0, y1, n) > design->cut) != (y1 >= cut[y0])) {
                    set_error("internal: pooled z rejection region is not monotone in y1");
                    return CSE_EUNSUPPORTED;
                }
        }
        // the calibration selection classifies outcomes by cut points on y1 per y0: S must not
        // increase with y1 for fixed y0 (so {y1 : S < s} is a suffix for every s)
        for (int y0 = 0; y0 <= n; ++y0)
            for (int y1 = 0; y1 < n; ++y1)
                if (S[y0 * n1 + y1 + 1] > S[y0 * n1 + y1]) {
                    set_error("internal: the 2-arm statistic is not monotone in y1");
                    return CSE_EUNSUPPORTED;
                }
        std::vector<int32_t> order(n1 * n1), group(n1 * n1);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return S[a] < S[b]; });
        std::vector<int32_t> pos(n1 * n1);
        for (int j = 0; j < n1 * n1; ++j) {
            group[j] = (j > 0 && S[order[j]] == S[order[j - 1]]) ? group[j - 1] : j;
            pos[order[j]] = j;
        }
        stage.add(&P->d_cut_tbl, cut.data(), cut.size());
        stage.add(&P->d_S_tbl, S.data(), S.size());
        stage.add(&P->d_S_order, order.data(), order.size());
        stage.add(&P->d_S_group, group.data(), group.size());
        stage.add(&P->d_S_pos, pos.data(), pos.size());
        // tie groups of S in ascending order: first position of each (and n1 * n1 after the
        // last), and per group g the cut vector cut_g(y0) = #{y1 : S(y0, y1) >= S_g}, so that
        // S < S_g iff y1 >= cut_g(y0); group n_groups has cut 0 (every outcome below it)
        {
            std::vector<int32_t> gstart;
            for (int j = 0; j < n1 * n1; ++j)
                if (group[j] == j) gstart.push_back(j);
            const int ng = (int)gstart.size();
            std::vector<uint8_t> gcut((size_t)(ng + 1) * n1, 0);
            for (int g = 0; g < ng; ++g) {
                const double Sg = S[order[gstart[g]]];
                for (int y0 = 0; y0 <= n; ++y0) {
                    int c = 0;
                    while (c <= n && S[y0 * n1 + c] >= Sg) ++c;
                    gcut[(size_t)g * n1 + y0] = (uint8_t)c;
                }
            }
            gstart.push_back(n1 * n1);
            P->n_groups = ng;
            stage.add(&P->d_gstart, gstart.data(), gstart.size());
            stage.add(&P->d_gcut, gcut.data(), gcut.size());
        }
    }

    for (int64_t t = 0; t < P->n_tiles; ++t)
        if (key_off[t] < 0) {
            set_error("internal: a tile was not placed in any batch");
            return CSE_EINVAL;
        }

    // ---- work items (launch shapes; cse_autotune may rebuild them) ----
    for (int64_t b = 0; b < P->n_blocks; ++b) P->block_sims += blk_sims[b];
    if (P->n_blocks > 0)
        if (int e = plan_work_items(P, P->tune_waves)) return e;
    // default workgroup counts (measured against cse_autotune): the 2-arm kernel's workgroups
    // hold 16 waves, the 4-arm kernels' 4
    if (kind == CSE_BINOM2_Z) P->tune_wgs = 2048;
    if (kind == CSE_BINOM2_Z || kind == CSE_HIER4 || kind == CSE_BASKET4)
        if (int e = plan_group_items(P, P->tune_wgs)) return e;

    stage.add(&P->d_theta, P->tile_theta.data(), P->tile_theta.size());
    stage.add(&P->d_N, P->tile_N.data(), P->tile_N.size());
    stage.add(&P->d_vert_off, P->vert_off.data(), P->vert_off.size());
    stage.add(&P->d_verts, P->verts.data(), P->verts.size());
    stage.add(&P->d_radii, P->tile_radii.data(), P->tile_radii.size());
    stage.add(&P->d_is_box, P->tile_is_box.data(), P->tile_is_box.size());
    stage.add(&P->d_in_null, P->tile_in_null.data(), P->tile_in_null.size());
    stage.add(&P->d_key_off, key_off.data(), key_off.size());
    stage.add(&P->d_key_stride, key_stride.data(), key_stride.size());
    // N classes for the Clopper-Pearson table
    {
        std::vector<int32_t> cls(P->tile_N.begin(), P->tile_N.end());
        std::sort(cls.begin(), cls.end());
        cls.erase(std::unique(cls.begin(), cls.end()), cls.end());
        std::vector<int64_t> off(cls.size()), base(P->n_tiles);
        int64_t e = 0;
        for (size_t c = 0; c < cls.size(); ++c) {
            off[c] = e;
            e += (int64_t)cls[c] + 1;
            P->max_cls_N = std::max(P->max_cls_N, cls[c]);
        }
        for (int64_t t = 0; t < P->n_tiles; ++t)
            base[t] = off[std::lower_bound(cls.begin(), cls.end(), P->tile_N[t]) - cls.begin()];
        P->n_cls = (int32_t)cls.size();
        P->n_cp = e;
        stage.add(&P->d_cls_N, cls.data(), cls.size());
        stage.add(&P->d_cls_off, off.data(), off.size());
        stage.add(&P->d_cp_base, base.data(), base.size());
        if (int r = stage.flush(P)) return r;
        if (kind == CSE_PHASE23) P->p23.key_off = P->d_key_off;
        CSE_HIP_TRY(hipMalloc((void **)&P->d_cp_mark, (size_t)e * sizeof(uint32_t)));
        CSE_HIP_TRY(hipMalloc((void **)&P->d_cp_tbl, (size_t)e * sizeof(double)));
    }
    const size_t nt = (size_t)P->n_tiles;
    CSE_HIP_TRY(hipMalloc((void **)&P->d_Rw, nt * sizeof(uint32_t)));
    // score sums: sum of T per arm; the Phase II/III design also sums the observed n per arm
    const size_t tw = (kind == CSE_PHASE23) ? 2 * (size_t)d : (size_t)d;
    CSE_HIP_TRY(hipMalloc((void **)&P->d_Tw, nt * tw * sizeof(unsigned long long)));
    CSE_HIP_TRY(hipMalloc((void **)&P->d_Zw, nt * sizeof(unsigned long long)));
    CSE_HIP_TRY(hipMalloc((void **)&P->d_apw, nt * sizeof(double)));
    CSE_HIP_TRY(hipMalloc((void **)&P->d_kw, nt * sizeof(int32_t)));
    CSE_HIP_TRY(hipMalloc((void **)&P->d_lamw, nt * sizeof(double)));
    CSE_HIP_TRY(hipMalloc((void **)&P->d_lamg, sizeof(double)));
    CSE_HIP_TRY(hipMalloc((void **)&P->d_minpart, 2 * MIN_PARTS * sizeof(double)));
    if (kind == CSE_BINOM2_Z) {
        CSE_HIP_TRY(hipMalloc((void **)&P->d_b2cut, (size_t)P->n_blocks * B2U * (NP35 + 1) * sizeof(uint4)));
        CSE_HIP_TRY(hipMalloc((void **)&P->d_b2br, nt * sizeof(int2)));
        CSE_HIP_TRY(hipMalloc((void **)&P->d_b2fb, (nt + 1) * sizeof(uint32_t)));
    }
    CSE_HIP_TRY(take_side_stream(P->device, &P->side));
    for (hipEvent_t *e : {&P->ev_sim, &P->ev_val, &P->ev_fork, &P->ev_inv})
        CSE_HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    return CSE_OK;
}

// Work items of the one-wave-per-block kernels: each block's simulations split into slices of
// whole 64-simulation chunks so that the grid has about target_waves waves.
int plan_work_items(Platten *P, int64_t target_waves) {
    std::vector<WorkItem> items;
    const int64_t slices = std::max<int64_t>(1, (target_waves + P->n_blocks - 1) / P->n_blocks);
    for (int64_t b = 0; b < P->n_blocks; ++b) {
        const int64_t N = P->blk_sims[b];
        const int64_t chunks = (N + WAVE - 1) / WAVE;
        const int64_t per = std::max<int64_t>(1, (chunks + slices - 1) / slices) * WAVE;
        for (int64_t k0 = 0; k0 < N; k0 += per) {
            WorkItem w{};
            w.blk = (int32_t)b;
            w.k_begin = (uint32_t)k0;
            w.k_end = (uint32_t)std::min<int64_t>(N, k0 + per);
            items.push_back(w);
        }
    }
    P->shape_gen->fetch_add(1);   // plans captured on the old arrays become stale
    if (P->d_items) CSE_HIP_TRY(hipFree(P->d_items));
    P->d_items = nullptr;
    P->n_items = (int64_t)items.size();
    P->tune_waves = target_waves;
    return upload(&P->d_items, items.data(), items.size());
}

// Workgroup items of the 2-arm and 4-arm kernels: groups of 4 consecutive blocks of equal N
// (blocks are ordered by N) whose four waves share the Philox words of a simulation range;
// ranges sliced so that the grid has about target_wgs workgroups.
// The candidate regions of the bracketed 4-arm calibration, sized for the current item ranges:
// allocated while the platten asks for that calibration (and its blocks' key rows fit the
// fused pass's LDS counters), freed otherwise.
int h4_regions(Platten *P) {
    const bool want = P->design.kind == CSE_HIER4 && P->h4_bracket && P->h4_max_rows <= H4_BROWS;
    const size_t nt = (size_t)std::max<int64_t>(P->n_tiles, 1);
    const size_t n_cnt = want ? nt * (size_t)(P->h4_maxs + 1) : 0, n_cand = want ? nt * (size_t)P->h4_tot : 0;
    if (n_cnt == P->h4_cnt_alloc && n_cand == P->h4_cand_alloc) return CSE_OK;
    if (P->d_h4cnt) CSE_HIP_TRY(hipFree(P->d_h4cnt));
    if (P->d_h4cand) CSE_HIP_TRY(hipFree(P->d_h4cand));
    P->d_h4cnt = nullptr;
    P->d_h4cand = nullptr;
    P->h4_cnt_alloc = P->h4_cand_alloc = 0;
    if (!want) return CSE_OK;
    if (hipMalloc((void **)&P->d_h4cnt, n_cnt * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&P->d_h4cand, n_cand * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        if (P->d_h4cnt) (void)hipFree(P->d_h4cnt);
        P->d_h4cnt = nullptr;
        P->d_h4cand = nullptr;
        set_error("cannot allocate the bracketed calibration's candidate regions");
        return CSE_ENOMEM;
    }
    P->h4_cnt_alloc = n_cnt;
    P->h4_cand_alloc = n_cand;
    return CSE_OK;
}

int plan_group_items(Platten *P, int64_t target_wgs) {
    std::vector<std::vector<int64_t>> groups;   // up to 4 (16 for the 2-arm design) blocks each (-1: none)
    const bool sq2 = P->design.kind == CSE_BINOM2_Z;
    if (sq2) {
        // 4 x 4 squares of blocks of equal N: block (row r, column c) goes to position
        // 4 (r & 3) + (c & 3) of square (r >> 2, c >> 2); a second block with the same
        // coordinates (two tiles at one grid point) opens another square
        std::map<std::tuple<int64_t, int64_t, int64_t, int64_t>, std::vector<int64_t>> sq;
        for (int64_t b = 0; b < P->n_blocks; ++b) {
            const int64_t r = P->blk_row[b], c = P->blk_col[b];
            const int pos = (int)(((r & (SQ2 - 1)) * SQ2) | (c & (SQ2 - 1)));
            for (int64_t dup = 0;; ++dup) {
                auto &g = sq[std::make_tuple(P->blk_sims[b], r / SQ2, c / SQ2, dup)];
                if (g.empty()) g.assign(SQ2W, -1);
                if (g[pos] < 0) {
                    g[pos] = b;
                    break;
                }
            }
        }
        for (auto &kv : sq) groups.push_back(kv.second);
    } else {
        for (int64_t b = 0; b < P->n_blocks; ++b) {
            if (groups.empty() || groups.back().size() == 4 || P->blk_sims[groups.back()[0]] != P->blk_sims[b])
                groups.push_back({});
            groups.back().push_back(b);
        }
    }
    const int64_t ng = (int64_t)groups.size();
    int64_t slices = std::max<int64_t>(1, (target_wgs + ng - 1) / ng);
    if (P->design.kind == CSE_HIER4) slices = std::min<int64_t>(slices, H4_MAXS);
    // at least 4 chunks of 64 simulations per item: an item's fixed work (thresholds, the final
    // transposes and atomics) then stays small beside its simulations
    constexpr int64_t MIN_ITEM_CHUNKS = 4;
    std::vector<GroupItem> gi, gpil;
    std::vector<SquareItem> si;
    int64_t gs = 0;
    int32_t maxs = 0, caps = 64;
    for (auto &g : groups) {
        int64_t first = -1;
        for (int64_t b : g)
            if (b >= 0 && first < 0) first = b;
        const int64_t N = P->blk_sims[first];
        const int64_t chunks = (N + WAVE - 1) / WAVE;
        const int64_t per = std::max<int64_t>(MIN_ITEM_CHUNKS, (chunks + slices - 1) / slices) * WAVE;
        if (!sq2) {
            // bracketed keys: the pilot's ranges, and room for twice the candidates an item range
            // expects (the bracket holds at most SEL_FILL_H4 of H4_SELCAND keys of the tile on
            // average) plus 32
            maxs = std::max<int32_t>(maxs, (int32_t)((N + per - 1) / per));
            if (N > H4_PILOT) {
                const double expect = 0.45 * 4096.0 * (double)std::min<int64_t>(per, N) / (double)N;
                caps = std::max<int32_t>(caps, (int32_t)((2.0 * expect + 32.0 + 31.0) / 32.0) * 32);
            }
            const int64_t np = std::min<int64_t>(N, H4_PILOT);
            const int64_t pper = std::max<int64_t>(MIN_ITEM_CHUNKS * WAVE, std::min<int64_t>(per, 4 * WAVE));
            for (int64_t k0 = 0; k0 < np; k0 += pper) {
                GroupItem it{};
                for (int w = 0; w < 4; ++w) it.blk[w] = w < (int)g.size() ? (int32_t)g[w] : -1;
                it.k_begin = (uint32_t)k0;
                it.k_end = (uint32_t)std::min<int64_t>(np, k0 + pper);
                it.slice = -1;
                gpil.push_back(it);
            }
        }
        int32_t slice = 0;
        for (int64_t k0 = 0; k0 < N; k0 += per) {
            const uint32_t kb = (uint32_t)k0, ke = (uint32_t)std::min<int64_t>(N, k0 + per);
            gs += (int64_t)(ke - kb);
            if (sq2) {
                SquareItem it{};
                for (int w = 0; w < SQ2W; ++w) it.blk[w] = w < (int)g.size() ? (int32_t)g[w] : -1;
                it.k_begin = kb;
                it.k_end = ke;
                si.push_back(it);
            } else {
                GroupItem it{};
                for (int w = 0; w < 4; ++w) it.blk[w] = w < (int)g.size() ? (int32_t)g[w] : -1;
                it.k_begin = kb;
                it.k_end = ke;
                it.slice = slice++;
                gi.push_back(it);
            }
        }
    }
    if (P->design.kind == CSE_HIER4) {
        if (P->d_gitems_pilot) CSE_HIP_TRY(hipFree(P->d_gitems_pilot));
        P->d_gitems_pilot = nullptr;
        P->n_gitems_pilot = (int64_t)gpil.size();
        if (!gpil.empty())
            if (int e = upload(&P->d_gitems_pilot, gpil.data(), gpil.size())) return e;
        P->h4_maxs = maxs;
        P->h4_caps = caps;
        P->h4_tot = (int64_t)H4_PCAP + (int64_t)maxs * caps;
        if (int e = h4_regions(P)) return e;
    }
    P->shape_gen->fetch_add(1);   // plans captured on the old arrays become stale
    if (P->d_gitems) CSE_HIP_TRY(hipFree(P->d_gitems));
    if (P->d_sqitems) CSE_HIP_TRY(hipFree(P->d_sqitems));
    P->d_gitems = nullptr;
    P->d_sqitems = nullptr;
    P->n_gitems = (int64_t)(sq2 ? si.size() : gi.size());
    P->group_sims = gs;
    P->tune_wgs = target_wgs;
    if (sq2) return upload(&P->d_sqitems, si.data(), si.size());
    return upload(&P->d_gitems, gi.data(), gi.size());
}

// Queue items of the Phase II/III kernel: (tile, `chunk` consecutive trials); the persistent
// grid has `grid` workgroups (-1: enough to fill the chip, at most one per 4 items).
int plan_queue_items(Platten *P, int32_t chunk, int64_t grid) {
    std::vector<WorkItem> items;
    P->p23_item_off.clear();
    for (int64_t t = 0; t < P->n_tiles; ++t) {
        P->p23_item_off.push_back((int64_t)items.size());
        for (int64_t k0 = 0; k0 < P->tile_N[t]; k0 += chunk) {
            WorkItem w{};
            w.blk = (int32_t)t;
            w.k_begin = (uint32_t)k0;
            w.k_end = (uint32_t)std::min<int64_t>(P->tile_N[t], k0 + chunk);
            items.push_back(w);
        }
    }
    P->p23_item_off.push_back((int64_t)items.size());
    P->shape_gen->fetch_add(1);   // plans captured on the old arrays become stale
    if (P->d_p23items) CSE_HIP_TRY(hipFree(P->d_p23items));
    P->d_p23items = nullptr;
    if (int e = upload(&P->d_p23items, items.data(), items.size())) return e;
    P->p23_chunk = chunk;
    P->p23.items = P->d_p23items;
    P->p23.n_items = (int64_t)items.size();
    const int64_t full = std::max<int64_t>(1, (P->p23.n_items + 3) / 4);
    P->p23_grid = grid > 0 ? std::min<int64_t>(grid, full) : std::min<int64_t>(full, 2048);
    return CSE_OK;
}

void free_platten(Platten *P) {
    if (!P) return;
    if (P->shape_gen) P->shape_gen->store(PLATTEN_GONE);   // plans on this platten refuse to replay
    (void)hipDeviceSynchronize();
    void *ptrs[] = {P->d_theta, P->d_N,    P->d_vert_off, P->d_verts,   P->d_key_off,
                    P->d_blocks, P->d_items, P->d_gitems, P->d_cut_tbl, P->d_S_tbl,  P->d_S_order,
                    P->d_S_group, P->d_keys, P->d_Rw,      P->d_Tw,     P->d_Zw,
                    P->d_apw,    P->d_kw,    P->d_lamw,    P->d_lamg,   P->d_cls_N,
                    P->d_cls_off, P->d_cp_base, P->d_cp_mark, P->d_cp_tbl,  P->d_radii,
                    P->d_is_box, P->d_key_stride, P->d_h4tbl, P->d_tileT, P->d_cfg,
                    P->d_queue,  P->d_p23items, P->d_gh, P->d_p23stats, P->d_p23look1, P->d_hnodes,
                    P->d_h4mask, P->d_S_pos, P->d_b2br, P->d_b2fb, P->d_b2cut, P->d_minpart, P->d_gstart, P->d_gcut, P->d_sqitems,
                    P->d_gitems_pilot, P->d_h4brk, P->d_h4below, P->d_h4cnt, P->d_h4cand, P->d_h4fb};
    auto in_arena = [&](void *q) {
        for (auto &a : P->arenas)
            if ((unsigned char *)q >= (unsigned char *)a.first && (unsigned char *)q < (unsigned char *)a.first + a.second)
                return true;
        return false;
    };
    for (void *q : ptrs)
        if (q && !in_arena(q)) (void)hipFree(q);
    for (auto &a : P->arenas) (void)hipFree(a.first);
    P->arenas.clear();
    for (hipEvent_t e : {P->ev_sim, P->ev_val, P->ev_fork, P->ev_inv})
        if (e) (void)hipEventDestroy(e);
    if (P->side) give_side_stream(P->device, P->side);
    P->side = nullptr;
}

}  // namespace cse
