// api.hip -- the extern "C" entry points of libcse.so (declared in include/cse.h).
#include <math.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cse_internal.h"
#include "kernels.h"

struct cse_platten {
    cse::Platten P;
};

// Calibration key workspace of cse_calibrate_noalloc: compiled into the library, one copy per
// device (resident from the library's first use on that device until the process ends).  In host
// code this name is a host-side handle, not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device (noalloc_workspace below).
static __device__ __align__(256) unsigned char scratch[(size_t)CSE_NOALLOC_SCRATCH_BYTES];

struct cse_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    int64_t n_nodes = 0;
    // the platten's launch-shape generation at capture: the graph's kernel arguments point into
    // that generation's work-item arrays, so the plan replays only while it is unchanged
    std::shared_ptr<std::atomic<uint64_t>> shape_gen;
    uint64_t gen_at_capture = 0;
};

namespace {

using cse::set_error;

#define CSE_LAUNCH(expr)                                                                   \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) {                                                            \
            set_error(std::string("launch failed: ") + hipGetErrorString(_e));             \
            return CSE_EHIP;                                                               \
        }                                                                                  \
    } while (0)

int check_handle(const cse_platten *h, const char *fn) {
    if (!h) {
        set_error(std::string(fn) + ": NULL platten");
        return CSE_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->P.device) {
        set_error(std::string(fn) + ": the current HIP device is not the platten's device");
        return CSE_EINVAL;
    }
    return CSE_OK;
}

bool in_unit(double x) { return x > 0.0 && x < 1.0; }

// Device address of `scratch` per device, looked up on the first cse_calibrate_noalloc call with
// that device current (no allocation: the array exists once the library's code is loaded there).
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int noalloc_workspace(int dev, void **out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("cse_calibrate_noalloc: device index outside the static workspace table");
        return CSE_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("cse_calibrate_noalloc: hipGetSymbolAddress of the static workspace failed: ") +
                      hipGetErrorString(e));
            return CSE_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CSE_OK;
}

// score_Z is the z-test's score sum; the binomial designs give score_T.
int check_scores(const cse::Platten &P, const void *score_T, const void *score_Z, const void *grad,
                 const char *fn) {
    (void)score_T;
    (void)grad;
    if (P.design.kind != CSE_ZTEST1 && score_Z) {
        set_error(std::string(fn) + ": score_Z is the z-test's score sum (CSE_ZTEST1 only)");
        return CSE_EUNSUPPORTED;
    }
    return CSE_OK;
}

// ---- launch timing (cse_profile_*) ----
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<int64_t, double>> g_totals;

hipEvent_t pool_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

thread_local bool t_capturing = false;   // no timing events inside a graph capture

struct Timed {
    ProfRec rec{};
    hipStream_t st;
    bool on = false;
    Timed(const char *name, hipStream_t s) : st(s) {
        if (t_capturing) return;
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (!g_prof_on) return;
        rec.name = name;
        rec.a = pool_event();
        rec.b = pool_event();
        if (!rec.a || !rec.b) return;
        on = hipEventRecord(rec.a, st) == hipSuccess;
    }
    ~Timed() {
        if (!on) return;
        std::lock_guard<std::mutex> g(g_prof_mu);
        if (hipEventRecord(rec.b, st) == hipSuccess) g_pending.push_back(rec);
    }
};

void prof_collect() {
    for (auto &r : g_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto &t = g_totals[r.name];
            t.first += 1;
            t.second += ms;
        }
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_pending.clear();
}

// Simulation with the design's fixed rule into the workspaces (R, score sums) and, when `keys` is not
// NULL, the calibration keys into `keys` (n_keys entries laid out as the platten's key offsets say).
// The 4-arm designs form score sums only when `scores` is set (they cost that kernel extra work);
// the others always do.
int run_sim(const cse::Platten &P, uint64_t seed, void *keys, hipStream_t st, bool scores = false) {
    CSE_LAUNCH(cse::launch_zero(P.d_Rw, P.n_tiles * sizeof(uint32_t), st));
    if (P.family == cse::FAM_NORMAL) {
        CSE_LAUNCH(cse::launch_zero(P.d_Zw, P.n_tiles * sizeof(unsigned long long), st));
        Timed tm(keys ? "ztest1_calib" : "ztest1", st);
        CSE_LAUNCH(cse::launch_ztest1(P, seed, P.d_Rw, P.d_Zw, (float *)keys, st));
    } else if (P.design.kind == CSE_HIER4 || P.design.kind == CSE_BASKET4) {
        const bool bk = P.design.kind == CSE_BASKET4;
        if (scores) CSE_LAUNCH(cse::launch_zero(P.d_Tw, P.n_tiles * P.d * sizeof(unsigned long long), st));
        Timed tm(keys ? (bk ? "basket4_calib" : "hier4_calib") : (bk ? "basket4" : "hier4"), st);
        CSE_LAUNCH(cse::launch_hier4(P, seed, P.d_Rw, scores ? P.d_Tw : nullptr, (float *)keys, st));
    } else if (P.design.kind == CSE_PHASE23) {
        CSE_LAUNCH(cse::launch_zero(P.d_Tw, P.n_tiles * 2 * P.d * sizeof(unsigned long long), st));
        Timed tm(keys ? "phase23_calib" : "phase23", st);
        CSE_LAUNCH(cse::launch_phase23(P, seed, P.d_Rw, P.d_Tw, (float *)keys, st));
    } else {
        CSE_LAUNCH(cse::launch_zero(P.d_Tw, P.n_tiles * P.d * sizeof(unsigned long long), st));
        Timed tm(keys ? "binom2_calib" : "binom2", st);
        CSE_LAUNCH(cse::launch_binom2(P, seed, P.d_Rw, P.d_Tw, (uint4 *)keys, st));
    }
    return CSE_OK;
}

// The 4-arm calibration with bracketed keys: pilot pass (float32 keys of the first H4_PILOT
// simulations), brackets once k is known (k_ready: the event after which it is, or null when
// it already is on st), then the pass over the other simulations (bracketed keys).  R and the
// score sums cover every simulation, as run_sim's.
int run_sim_h4(const cse::Platten &P, uint64_t seed, void *keys, hipStream_t st, bool scores, hipEvent_t k_ready,
               const int32_t *kk, double *lam, int32_t *rej_at) {
    CSE_LAUNCH(cse::launch_zero(P.d_Rw, P.n_tiles * sizeof(uint32_t), st));
    if (scores) CSE_LAUNCH(cse::launch_zero(P.d_Tw, P.n_tiles * P.d * sizeof(unsigned long long), st));
    unsigned long long *sT = scores ? P.d_Tw : nullptr;
    {
        Timed tm("hier4_pilot", st);
        CSE_LAUNCH(cse::launch_hier4(P, seed, P.d_Rw, sT, (float *)keys, st, cse::H4_PASS_PILOT));
    }
    if (k_ready) CSE_HIP_TRY(hipStreamWaitEvent(st, k_ready, 0));
    {
        Timed tm("h4_bracket", st);
        CSE_LAUNCH(cse::launch_h4_bracket(P, (const float *)keys, kk, lam, rej_at, st));
    }
    Timed tm("hier4_calib", st);
    CSE_LAUNCH(cse::launch_hier4(P, seed, P.d_Rw, sT, nullptr, st, cse::H4_PASS_MAIN));
    return CSE_OK;
}

size_t key_bytes(const cse::Platten &P) {
    const size_t esz = (P.design.kind == CSE_BINOM2_Z) ? cse::REC2_BYTES : 4;
    return (size_t)P.n_keys * esz;
}

int ensure_keys(cse::Platten &P) {
    const size_t need = key_bytes(P);
    if (P.d_keys && P.keys_bytes >= need) return CSE_OK;
    if (P.d_keys) {
        (void)hipFree(P.d_keys);
        P.d_keys = nullptr;
    }
    if (hipMalloc(&P.d_keys, need) != hipSuccess) {
        (void)hipGetLastError();
        set_error("cse_calibrate: cannot allocate the calibration key workspace");
        return CSE_ENOMEM;
    }
    P.keys_bytes = need;
    return CSE_OK;
}

int check_validate(const cse_platten *p, double delta, const void *score_T, const void *score_Z, const void *grad,
                   const double *tile_bound, const char *fn) {
    if (int e = check_handle(p, fn)) return e;
    if (!in_unit(delta)) {
        set_error(std::string(fn) + ": delta must lie in (0, 1)");
        return CSE_EINVAL;
    }
    if (!tile_bound) {
        set_error(std::string(fn) + ": tile_bound must not be NULL");
        return CSE_EINVAL;
    }
    return check_scores(p->P, score_T, score_Z, grad, fn);
}

int check_calibrate(const cse_platten *p, double alpha, double delta, const void *score_T, const void *score_Z,
                    const void *grad, bool want_bound, const char *fn) {
    if (int e = check_handle(p, fn)) return e;
    if (!in_unit(alpha)) {
        set_error(std::string(fn) + ": alpha must lie in (0, 1)");
        return CSE_EINVAL;
    }
    if (want_bound && !in_unit(delta)) {
        set_error(std::string(fn) + ": delta must lie in (0, 1) when cp_upper or tile_bound is requested");
        return CSE_EINVAL;
    }
    return check_scores(p->P, score_T, score_Z, grad, fn);
}

// Validation (Algorithm 1) on stream st: simulate with the design's fixed rule, then the
// Clopper-Pearson + Tilt-Bound of every tile.  Arguments checked by the caller.
int validate_impl(const cse::Platten &P, uint64_t seed, double delta, int32_t *reject, int64_t *score_T,
                  double *score_Z, double *grad, double *cp_upper, double *tile_bound, double *q_star,
                  hipStream_t st) {
    if (int e = run_sim(P, seed, nullptr, st, score_T || grad)) return e;
    CSE_LAUNCH(cse::launch_finish(P, P.d_Rw, P.d_Tw, P.d_Zw, reject, score_T, score_Z, grad, st));
    Timed tm("bound_validate", st);
    CSE_LAUNCH(cse::launch_bound(P, 0, P.d_Rw, nullptr, delta, tile_bound, q_star, nullptr, cp_upper, st));
    return CSE_OK;
}

// Calibration (Algorithm 2) on stream st with the key workspace `keys` (key_bytes(P) bytes).
int calibrate_impl(const cse::Platten &P, void *keys, uint64_t seed, double alpha, double *alpha_prime, int32_t *k,
                   double *lambda_tile, double *lambda_global, int32_t *reject_at_lambda, double delta,
                   int32_t *reject, int64_t *score_T, double *score_Z, double *grad, double *cp_upper,
                   double *tile_bound, hipStream_t st, bool full_keys = false) {
    double *ap = alpha_prime ? alpha_prime : P.d_apw;
    // 4-arm design: bracketed keys when the platten asks for them (CSE_OPT_H4_BRACKET) and every key
    // need not reach HBM (the randomised tie-break reads them)
    const bool h4b = P.design.kind == CSE_HIER4 && !full_keys && P.h4_bracket && P.d_h4cand;
    int32_t *kk = k ? k : P.d_kw;
    double *lam = lambda_tile ? lambda_tile : P.d_lamw;
    // The step's dependencies: alpha' -> k -> selection; simulation -> selection, finish and
    // the validation bound.  The fused simulation runs alone (it fills the chip); afterwards
    // the validation bound (float64, latency-bound) runs on the side stream beside the
    // selection, forked from and joined into `st` by events.  Captured as a graph, the
    // inversion and the 2-arm brackets (which do not depend on the simulation) are a branch
    // beside the simulation too; eager calls keep them in line, so that every kernel's own
    // timing describes that kernel alone.
    // target level of each tile (Section 7.2), then its order-statistic index (Section 7.1)
    const bool branch_invert = t_capturing;
    {
        hipStream_t is = branch_invert ? P.side : st;
        if (branch_invert) {
            CSE_HIP_TRY(hipEventRecord(P.ev_fork, st));
            CSE_HIP_TRY(hipStreamWaitEvent(is, P.ev_fork, 0));
        }
        {
            Timed tm("bound_invert", is);
            CSE_LAUNCH(cse::launch_bound(P, 1, nullptr, nullptr, alpha, ap, nullptr, kk, nullptr, is));
        }
        if (P.design.kind == CSE_BINOM2_Z) {   // the selection's brackets need k only
            Timed tm("b2_bracket", is);
            CSE_LAUNCH(cse::launch_b2_bracket(P, kk, is));
        }
        if (branch_invert) CSE_HIP_TRY(hipEventRecord(P.ev_inv, is));
    }
    if (h4b) {
        if (int e = run_sim_h4(P, seed, keys, st, score_T || grad, branch_invert ? P.ev_inv : nullptr, kk, lam,
                               reject_at_lambda))
            return e;
    } else if (int e = run_sim(P, seed, keys, st, score_T || grad)) {
        return e;
    }
    const bool want_bound = cp_upper || tile_bound;
    if (want_bound) {
        hipStream_t side = P.side;
        CSE_HIP_TRY(hipEventRecord(P.ev_sim, st));
        CSE_HIP_TRY(hipStreamWaitEvent(side, P.ev_sim, 0));
        // alpha' lives in the caller's buffer or in d_apw, and is no longer read once k is
        // known, so d_apw can hold the bound the caller did not ask for.
        double *tb = tile_bound ? tile_bound : P.d_apw;
        {
            Timed tm("bound_validate", side);
            CSE_LAUNCH(cse::launch_bound(P, 0, P.d_Rw, nullptr, delta, tb, nullptr, nullptr, cp_upper, side));
        }
        CSE_HIP_TRY(hipEventRecord(P.ev_val, side));
    }
    if (branch_invert) CSE_HIP_TRY(hipStreamWaitEvent(st, P.ev_inv, 0));   // k before the selection
    {
        Timed tm("select", st);
        if (h4b)
            CSE_LAUNCH(cse::launch_h4_select(P, seed, kk, lam, reject_at_lambda, st));
        else
            CSE_LAUNCH(cse::launch_select(P, keys, kk, lam, reject_at_lambda, st));
    }
    CSE_LAUNCH(cse::launch_min(P, lam, P.d_in_null, P.n_tiles, lambda_global ? lambda_global : P.d_lamg, st));
    if (reject || score_T || score_Z || grad)
        CSE_LAUNCH(cse::launch_finish(P, P.d_Rw, P.d_Tw, P.d_Zw, reject, score_T, score_Z, grad, st));
    if (want_bound) CSE_HIP_TRY(hipStreamWaitEvent(st, P.ev_val, 0));   // join
    return CSE_OK;
}

}  // namespace

extern "C" {

const char *cse_last_error(void) { return cse::get_error(); }

int cse_platten_create(const cse_design *design, int64_t n_boxes, const double *theta,
                       const double *radii, const int32_t *sims, int32_t flags, cse_platten **out) {
    if (!out) {
        set_error("cse_platten_create: NULL out");
        return CSE_EINVAL;
    }
    *out = nullptr;
    cse_platten *h = new (std::nothrow) cse_platten();
    if (!h) {
        set_error("cse_platten_create: out of host memory");
        return CSE_ENOMEM;
    }
    int e;
    try {
        e = cse::build_platten(design, n_boxes, theta, radii, sims, flags, &h->P);
    } catch (const std::bad_alloc &) {
        set_error("cse_platten_create: out of host memory");
        e = CSE_ENOMEM;
    } catch (...) {
        set_error("cse_platten_create: unexpected host exception");
        e = CSE_EINVAL;
    }
    if (e != CSE_OK) {
        cse::free_platten(&h->P);
        delete h;
        return e;
    }
    *out = h;
    return CSE_OK;
}

int cse_platten_destroy(cse_platten *p) {
    if (!p) return CSE_OK;
    cse::free_platten(&p->P);
    delete p;
    return CSE_OK;
}

int64_t cse_platten_size(const cse_platten *p) { return p ? p->P.n_tiles : -1; }

int cse_platten_tiles(const cse_platten *p, double *theta, double *radii) {
    if (!p) {
        set_error("cse_platten_tiles: NULL platten");
        return CSE_EINVAL;
    }
    const auto &P = p->P;
    const size_t n = (size_t)P.n_tiles * P.d;
    if (theta) std::copy(P.tile_theta.begin(), P.tile_theta.begin() + n, theta);
    if (radii) std::copy(P.tile_radii.begin(), P.tile_radii.begin() + n, radii);
    return CSE_OK;
}

int cse_platten_describe(const cse_platten *p, int64_t *box, int32_t *cfg, int32_t *n_vert,
                         int32_t *in_null) {
    if (!p) {
        set_error("cse_platten_describe: NULL platten");
        return CSE_EINVAL;
    }
    const auto &P = p->P;
    for (int64_t t = 0; t < P.n_tiles; ++t) {
        if (box) box[t] = P.tile_box[t];
        if (cfg) cfg[t] = P.tile_cfg[t];
        if (n_vert) n_vert[t] = P.tile_nv[t];
        if (in_null) in_null[t] = P.tile_in_null[t];
    }
    return CSE_OK;
}

int cse_simulate(const cse_platten *p, uint64_t seed, int32_t *reject, int64_t *score_T,
                 double *score_Z, double *grad, void *stream) {
    if (int e = check_handle(p, "cse_simulate")) return e;
    if (!reject) {
        set_error("cse_simulate: reject must not be NULL");
        return CSE_EINVAL;
    }
    const auto &P = p->P;
    if (int e = check_scores(P, score_T, score_Z, grad, "cse_simulate")) return e;
    hipStream_t st = (hipStream_t)stream;
    if (int e = run_sim(P, seed, nullptr, st, score_T || grad)) return e;
    CSE_LAUNCH(cse::launch_finish(P, P.d_Rw, P.d_Tw, P.d_Zw, reject, score_T, score_Z, grad, st));
    return CSE_OK;
}

int cse_validate(const cse_platten *p, uint64_t seed, double delta, int32_t *reject,
                 int64_t *score_T, double *score_Z, double *grad, double *cp_upper,
                 double *tile_bound, double *q_star, void *stream) {
    if (int e = check_validate(p, delta, score_T, score_Z, grad, tile_bound, "cse_validate")) return e;
    return validate_impl(p->P, seed, delta, reject, score_T, score_Z, grad, cp_upper, tile_bound, q_star,
                         (hipStream_t)stream);
}

int cse_calibrate(const cse_platten *p, uint64_t seed, double alpha, double *alpha_prime,
                  int32_t *k, double *lambda_tile, double *lambda_global,
                  int32_t *reject_at_lambda, double delta, int32_t *reject, int64_t *score_T,
                  double *score_Z, double *grad, double *cp_upper, double *tile_bound,
                  void *stream) {
    if (int e = check_calibrate(p, alpha, delta, score_T, score_Z, grad, cp_upper || tile_bound, "cse_calibrate"))
        return e;
    auto &P = const_cast<cse_platten *>(p)->P;
    if (int e = ensure_keys(P)) return e;
    return calibrate_impl(P, P.d_keys, seed, alpha, alpha_prime, k, lambda_tile, lambda_global, reject_at_lambda, delta,
                          reject, score_T, score_Z, grad, cp_upper, tile_bound, (hipStream_t)stream);
}

int cse_calibrate_noalloc(const cse_platten *p, uint64_t seed, double alpha, double *alpha_prime, int32_t *k,
                          double *lambda_tile, double *lambda_global, int32_t *reject_at_lambda, double delta,
                          int32_t *reject, int64_t *score_T, double *score_Z, double *grad, double *cp_upper,
                          double *tile_bound, void *stream) {
    if (int e = check_calibrate(p, alpha, delta, score_T, score_Z, grad, cp_upper || tile_bound,
                                "cse_calibrate_noalloc"))
        return e;
    const auto &P = p->P;
    const size_t need = key_bytes(P);
    if (need > (size_t)CSE_NOALLOC_SCRATCH_BYTES) {
        set_error("cse_calibrate_noalloc: the platten's calibration keys need " + std::to_string(need) +
                  " bytes, more than the static workspace of " + std::to_string((long long)CSE_NOALLOC_SCRATCH_BYTES) +
                  " bytes (use cse_calibrate)");
        return CSE_EINVAL;
    }
    void *ws = nullptr;
    if (int e = noalloc_workspace(P.device, &ws)) return e;
    return calibrate_impl(P, ws, seed, alpha, alpha_prime, k, lambda_tile, lambda_global, reject_at_lambda, delta,
                          reject, score_T, score_Z, grad, cp_upper, tile_bound, (hipStream_t)stream);
}

// ---- plans: one validation or calibration step captured into a HIP graph ----
namespace {
int capture_plan(const cse_platten *p, const std::function<int(hipStream_t)> &body, cse_plan **out,
                 const char *fn) {
    if (!out) {
        set_error(std::string(fn) + ": NULL out");
        return CSE_EINVAL;
    }
    *out = nullptr;
    hipStream_t cs = nullptr;
    CSE_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    int e = CSE_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        set_error(std::string(fn) + ": hipStreamBeginCapture failed");
        e = CSE_EHIP;
    } else {
        t_capturing = true;
        e = body(cs);
        t_capturing = false;
        const hipError_t ee = hipStreamEndCapture(cs, &g);
        if (e == CSE_OK && ee != hipSuccess) {
            set_error(std::string(fn) + ": hipStreamEndCapture failed: " + hipGetErrorString(ee));
            e = CSE_EHIP;
        }
    }
    hipGraphExec_t ex = nullptr;
    if (e == CSE_OK && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        set_error(std::string(fn) + ": hipGraphInstantiate failed");
        e = CSE_EHIP;
    }
    (void)hipStreamDestroy(cs);
    if (e != CSE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    cse_plan *pl = new (std::nothrow) cse_plan();
    if (!pl) {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
        set_error(std::string(fn) + ": out of host memory");
        return CSE_ENOMEM;
    }
    pl->graph = g;
    pl->exec = ex;
    pl->device = p->P.device;
    pl->shape_gen = p->P.shape_gen;
    pl->gen_at_capture = p->P.shape_gen->load();
    pl->n_nodes = 0;
    size_t nn = 0;
    if (hipGraphGetNodes(g, nullptr, &nn) == hipSuccess) pl->n_nodes = (int64_t)nn;
    *out = pl;
    return CSE_OK;
}
}  // namespace

int cse_plan_validate(const cse_platten *p, uint64_t seed, double delta, int32_t *reject, int64_t *score_T,
                      double *score_Z, double *grad, double *cp_upper, double *tile_bound, double *q_star,
                      cse_plan **out) {
    if (int e = check_validate(p, delta, score_T, score_Z, grad, tile_bound, "cse_plan_validate")) return e;
    const auto &P = p->P;
    return capture_plan(p, [&](hipStream_t cs) {
        return validate_impl(P, seed, delta, reject, score_T, score_Z, grad, cp_upper, tile_bound, q_star, cs);
    }, out, "cse_plan_validate");
}

int cse_plan_calibrate(const cse_platten *p, uint64_t seed, double alpha, double *alpha_prime, int32_t *k,
                       double *lambda_tile, double *lambda_global, int32_t *reject_at_lambda, double delta,
                       int32_t *reject, int64_t *score_T, double *score_Z, double *grad, double *cp_upper,
                       double *tile_bound, cse_plan **out) {
    if (int e = check_calibrate(p, alpha, delta, score_T, score_Z, grad, cp_upper || tile_bound,
                                "cse_plan_calibrate"))
        return e;
    auto &P = const_cast<cse_platten *>(p)->P;
    if (int e = ensure_keys(P)) return e;   // allocation stays outside the graph
    return capture_plan(p, [&](hipStream_t cs) {
        return calibrate_impl(P, P.d_keys, seed, alpha, alpha_prime, k, lambda_tile, lambda_global, reject_at_lambda, delta,
                              reject, score_T, score_Z, grad, cp_upper, tile_bound, cs);
    }, out, "cse_plan_calibrate");
}

int cse_plan_launch(const cse_plan *plan, void *stream) {
    if (!plan) {
        set_error("cse_plan_launch: NULL plan");
        return CSE_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) {
        set_error("cse_plan_launch: the current HIP device is not the plan's device");
        return CSE_EINVAL;
    }
    const uint64_t gen = plan->shape_gen ? plan->shape_gen->load() : cse::PLATTEN_GONE;
    if (gen != plan->gen_at_capture) {
        set_error(gen == cse::PLATTEN_GONE
                      ? "cse_plan_launch: the plan's platten has been destroyed"
                      : "cse_plan_launch: cse_autotune rebuilt the platten's launch shape after this plan was "
                        "captured; capture a new plan");
        return CSE_EINVAL;
    }
    CSE_HIP_TRY(hipGraphLaunch(plan->exec, (hipStream_t)stream));
    return CSE_OK;
}

int64_t cse_plan_nodes(const cse_plan *plan) { return plan ? plan->n_nodes : -1; }

int cse_autotune(cse_platten *p, uint64_t seed, int64_t max_trials, int64_t out[2], void *stream) {
    if (int e = check_handle(p, "cse_autotune")) return e;
    if (!out || max_trials < 1) {
        set_error("cse_autotune: NULL out or max_trials < 1");
        return CSE_EINVAL;
    }
    auto &P = p->P;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CSE_HIP_TRY(hipEventCreate(&e0));
    CSE_HIP_TRY(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    // mean time of `reps` launches of f after one untimed launch
    auto timeit = [&](const std::function<int()> &f, int reps, float *ms) -> int {
        if (int e = f()) return e;
        CSE_HIP_TRY(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r)
            if (int e = f()) return e;
        CSE_HIP_TRY(hipEventRecord(e1, st));
        CSE_HIP_TRY(hipEventSynchronize(e1));
        CSE_HIP_TRY(hipEventElapsedTime(ms, e0, e1));
        *ms /= (float)reps;
        return CSE_OK;
    };
    out[0] = out[1] = 0;
    if (P.design.kind == CSE_PHASE23) {
        // a strided sample of tiles holding at most max_trials trials
        int64_t total = P.total_sims, stride = std::max<int64_t>(1, (total + max_trials - 1) / max_trials);
        std::vector<int64_t> tiles;
        for (int64_t t = 0; t < P.n_tiles; t += stride) tiles.push_back(t);
        const int32_t chunks[4] = {64, 128, 256, 512};
        const int64_t grids[3] = {512, 1024, 2048};
        float best = 3.4e38f;
        int32_t bc = P.p23_chunk;
        int64_t bg = P.p23_grid;
        struct DevItems {   // the sample's item list, freed on every exit
            cse::WorkItem *p = nullptr;
            ~DevItems() {
                if (p) (void)hipFree(p);
            }
        } d_it;
        for (int32_t c : chunks) {
            std::vector<cse::WorkItem> items;
            for (int64_t t : tiles)
                for (int64_t k0 = 0; k0 < P.tile_N[t]; k0 += c) {
                    cse::WorkItem w{};
                    w.blk = (int32_t)t;
                    w.k_begin = (uint32_t)k0;
                    w.k_end = (uint32_t)std::min<int64_t>(P.tile_N[t], k0 + c);
                    items.push_back(w);
                }
            if (d_it.p) CSE_HIP_TRY(hipFree(d_it.p));
            d_it.p = nullptr;
            CSE_HIP_TRY(hipMalloc((void **)&d_it.p, items.size() * sizeof(cse::WorkItem)));
            CSE_HIP_TRY(hipMemcpy(d_it.p, items.data(), items.size() * sizeof(cse::WorkItem), hipMemcpyHostToDevice));
            const int64_t full = std::max<int64_t>(1, ((int64_t)items.size() + 3) / 4);
            for (int64_t g : grids) {
                const int64_t gg = std::min(g, full);
                float ms = 0.0f;
                if (int e = timeit([&]() -> int {
                        CSE_LAUNCH(cse::launch_phase23_items(P, seed, d_it.p, (int64_t)items.size(), gg, P.d_Rw, st));
                        return CSE_OK;
                    }, 1, &ms))
                    return e;
                if (ms < best) {
                    best = ms;
                    bc = c;
                    bg = g;
                }
            }
        }
        if (int e = cse::plan_queue_items(&P, bc, bg)) return e;
        out[0] = P.p23_chunk;
        out[1] = P.p23_grid;
        return CSE_OK;
    }
    // one-wave-per-block (z-test) or group kernels (2-arm, 4-arm): time the calibration launch
    if (int e = ensure_keys(P)) return e;
    const bool group = P.design.kind == CSE_BINOM2_Z || P.design.kind == CSE_HIER4 || P.design.kind == CSE_BASKET4;
    const int64_t cands[7] = {1024, 2048, 4096, 8192, 16384, 32768, 65536};
    const int64_t wave_cands[7] = {4096, 8192, 16384, 32768, 65536, 131072, 262144};
    float best = 3.4e38f;
    int64_t bv = group ? P.tune_wgs : P.tune_waves;
    for (int i = 0; i < 7; ++i) {
        const int64_t v = group ? cands[i] : wave_cands[i];
        if (int e = group ? cse::plan_group_items(&P, v) : cse::plan_work_items(&P, v)) return e;
        // the calibration launch (keys) and the validation launch (no keys) together: the
        // best shape of one need not be the best of the other
        float ms = 0.0f, ms_val = 0.0f;
        if (int e = timeit([&]() { return run_sim(P, seed, P.d_keys, st); }, 3, &ms)) return e;
        if (int e = timeit([&]() { return run_sim(P, seed, nullptr, st); }, 3, &ms_val)) return e;
        ms += ms_val;
        if (ms < best) {
            best = ms;
            bv = v;
        }
    }
    if (int e = group ? cse::plan_group_items(&P, bv) : cse::plan_work_items(&P, bv)) return e;
    out[0] = bv;
    return CSE_OK;
}

int cse_plan_destroy(cse_plan *plan) {
    if (!plan) return CSE_OK;
    (void)hipDeviceSynchronize();
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return CSE_OK;
}

int cse_bound(const cse_platten *p, int32_t mode, const int32_t *R, const double *a,
              double delta_or_alpha, double *out, double *q_star, void *stream) {
    if (int e = check_handle(p, "cse_bound")) return e;
    if (!out || mode < 0 || mode > 2) {
        set_error("cse_bound: NULL out or mode outside {0, 1, 2}");
        return CSE_EINVAL;
    }
    if (mode == 0 && !R) {
        set_error("cse_bound: mode 0 needs R");
        return CSE_EINVAL;
    }
    if (mode == 2 && !a) {
        set_error("cse_bound: mode 2 needs a");
        return CSE_EINVAL;
    }
    if (mode != 2 && !in_unit(delta_or_alpha)) {
        set_error("cse_bound: delta/alpha must lie in (0, 1)");
        return CSE_EINVAL;
    }
    const auto &P = p->P;
    CSE_LAUNCH(cse::launch_bound(P, mode, (const uint32_t *)R, a, delta_or_alpha, out, q_star,
                                 nullptr, nullptr, (hipStream_t)stream));
    return CSE_OK;
}

int cse_validate_lower(const cse_platten *p, const int32_t *R, double delta, double *cp_lower, double *lower,
                       double *q_star, void *stream) {
    if (int e = check_handle(p, "cse_validate_lower")) return e;
    if (!R || !lower) {
        set_error("cse_validate_lower: R and lower must not be NULL");
        return CSE_EINVAL;
    }
    if (!in_unit(delta)) {
        set_error("cse_validate_lower: delta must lie in (0, 1)");
        return CSE_EINVAL;
    }
    const auto &P = p->P;
    if (P.n_tiles == 0) return CSE_OK;
    hipStream_t st = (hipStream_t)stream;
    Timed tm("bound_lower", st);
    CSE_LAUNCH(cse::launch_bound(P, 3, (const uint32_t *)R, nullptr, delta, lower, q_star, nullptr, cp_lower, st));
    return CSE_OK;
}

int cse_confidence_set(const cse_platten *p, const double *s_obs, int64_t s_stride, const double *lambda_tile,
                       const double *coef, int32_t link, int32_t *keep, double *e_lo, double *e_hi,
                       double *e_range, void *stream) {
    if (int e = check_handle(p, "cse_confidence_set")) return e;
    if (!s_obs || !lambda_tile || !coef || !keep || !e_lo || !e_hi || !e_range) {
        set_error("cse_confidence_set: s_obs, lambda_tile, coef, keep, e_lo, e_hi and e_range must not be NULL");
        return CSE_EINVAL;
    }
    if (link != 0 && link != 1) {
        set_error("cse_confidence_set: link must be 0 (identity) or 1 (expit)");
        return CSE_EINVAL;
    }
    if (s_stride != 0 && s_stride != 1) {
        set_error("cse_confidence_set: s_stride must be 0 (one statistic for all tiles) or 1");
        return CSE_EINVAL;
    }
    const auto &P = p->P;
    for (int a = 0; a <= P.d; ++a)
        if (!std::isfinite(coef[a])) {
            set_error("cse_confidence_set: coefficients must be finite");
            return CSE_EINVAL;
        }
    hipStream_t st = (hipStream_t)stream;
    Timed tm("confidence_set", st);
    CSE_LAUNCH(cse::launch_confset(P, s_obs, s_stride, lambda_tile, coef, link, keep, e_lo, e_hi, e_range, st));
    return CSE_OK;
}

int cse_calibrate_tiebreak(const cse_platten *p, uint64_t seed, double alpha, double *alpha_prime, int32_t *k,
                           double *lambda_tile, uint32_t *u_tile, double *lambda_global, uint32_t *u_global,
                           int32_t *reject_at_lambda, void *stream) {
    if (int e = check_calibrate(p, alpha, 0.5, nullptr, nullptr, nullptr, false, "cse_calibrate_tiebreak")) return e;
    if (!lambda_tile || !u_tile || !lambda_global || !u_global || !reject_at_lambda) {
        set_error("cse_calibrate_tiebreak: lambda_tile, u_tile, lambda_global, u_global and reject_at_lambda "
                  "must not be NULL");
        return CSE_EINVAL;
    }
    auto &P = const_cast<cse_platten *>(p)->P;
    if (P.n_tiles == 0) {
        set_error("cse_calibrate_tiebreak: the platten has no tiles");
        return CSE_EINVAL;
    }
    if (int e = ensure_keys(P)) return e;
    hipStream_t st = (hipStream_t)stream;
    int32_t *kk = k ? k : P.d_kw;
    if (int e = calibrate_impl(P, P.d_keys, seed, alpha, alpha_prime, kk, lambda_tile, nullptr, reject_at_lambda, 0.5, nullptr,
                               nullptr, nullptr, nullptr, nullptr, nullptr, st, true))
        return e;
    {
        Timed tm("tiebreak", st);
        CSE_LAUNCH(cse::launch_tiebreak(P, seed, kk, lambda_tile, reject_at_lambda, u_tile, st));
    }
    CSE_LAUNCH(cse::launch_min_pair(P, lambda_tile, u_tile, P.d_in_null, P.n_tiles, lambda_global, u_global, st));
    return CSE_OK;
}

int cse_taylor(const cse_platten *p, const double *f, const double *grad, double *bound, int32_t *vertex,
               double *point, void *stream) {
    if (int e = check_handle(p, "cse_taylor")) return e;
    if (!f || !grad || !bound) {
        set_error("cse_taylor: f, grad and bound must not be NULL");
        return CSE_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    Timed tm("taylor", st);
    CSE_LAUNCH(cse::launch_taylor(p->P, f, grad, bound, vertex, point, st));
    return CSE_OK;
}

int cse_simulate_per_tile(const cse_platten *p, uint64_t seed, int64_t tile_begin, int64_t tile_end,
                          int32_t *reject, void *stream) {
    if (int e = check_handle(p, "cse_simulate_per_tile")) return e;
    const auto &P = p->P;
    if (!reject || tile_begin < 0 || tile_end > P.n_tiles || tile_begin > tile_end) {
        set_error("cse_simulate_per_tile: bad tile range or NULL reject");
        return CSE_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    CSE_LAUNCH(cse::launch_zero(reject + tile_begin, (tile_end - tile_begin) * sizeof(int32_t), st));
    for (int64_t t = tile_begin; t < tile_end; ++t) {
        Timed tm("plain_tile", st);
        if (P.design.kind == CSE_HIER4 || P.design.kind == CSE_BASKET4) {
            CSE_LAUNCH(cse::launch_hier4_plain(P, seed, t, (uint32_t *)(reject + t), st));
            continue;
        }
        if (P.design.kind == CSE_PHASE23) {
            CSE_LAUNCH(cse::launch_phase23_tile(P, seed, t, (uint32_t *)(reject + t), st));
            continue;
        }
        uint32_t T0 = 0, T1 = 0;
        if (P.family == cse::FAM_BINOM) {
            T0 = P.tile_T[t * 2];
            T1 = P.tile_T[t * 2 + 1];
        }
        CSE_LAUNCH(cse::launch_plain_tile(P, seed, t, T0, T1, (uint32_t *)(reject + t), st));
    }
    return CSE_OK;
}

int cse_platten_stats(const cse_platten *p, int64_t out[12]) {
    if (!p || !out) {
        set_error("cse_platten_stats: NULL argument");
        return CSE_EINVAL;
    }
    const auto &P = p->P;
    out[0] = P.n_tiles;
    out[1] = P.n_blocks;
    out[2] = P.n_items;
    out[3] = P.n_keys;
    out[4] = P.total_sims;
    out[5] = (P.family == cse::FAM_NORMAL) ? cse::B1T : cse::B2U * cse::B2V;
    out[6] = P.max_N;
    out[7] = P.block_sims;
    out[8] = P.group_sims;
    out[9] = P.n_cls;
    out[10] = (int64_t)(P.table_ms * 1000.0);
    out[11] = P.design.kind == CSE_PHASE23 ? P.p23_chunk
              : (P.design.kind == CSE_ZTEST1 ? P.tune_waves : P.tune_wgs);
    return CSE_OK;
}

int cse_platten_set_option(cse_platten *p, int32_t option, double value) {
    if (int e = check_handle(p, "cse_platten_set_option")) return e;
    if (option == CSE_OPT_H4_BRACKET) {
        if (value != 0.0 && value != 1.0) {
            set_error("cse_platten_set_option: CSE_OPT_H4_BRACKET takes 0 or 1");
            return CSE_EINVAL;
        }
        p->P.h4_bracket = value == 1.0;
        if (int e = cse::h4_regions(&p->P)) {   // the candidate regions live while the option is on
            p->P.h4_bracket = false;
            return e;
        }
        return CSE_OK;
    }
    if (option != CSE_OPT_B2_MARGIN && option != CSE_OPT_H4_MARGIN) {
        set_error("cse_platten_set_option: unknown option");
        return CSE_EINVAL;
    }
    if (!(value >= 0.0 && value <= 100.0)) {
        set_error("cse_platten_set_option: the bracket margin must lie in [0, 100]");
        return CSE_EINVAL;
    }
    if (option == CSE_OPT_B2_MARGIN)
        p->P.b2_margin = (float)value;
    else
        p->P.h4_margin = (float)value;
    return CSE_OK;
}

int cse_work_counters(const cse_platten *p, int64_t out[4], void *stream) {
    if (int e = check_handle(p, "cse_work_counters")) return e;
    const auto &P = p->P;
    if (!out) {
        set_error("cse_work_counters: NULL out");
        return CSE_EINVAL;
    }
    if (P.design.kind == CSE_BINOM2_Z || P.design.kind == CSE_HIER4) {   // tiles the last selection took exactly
        uint32_t n_fb = 0u;
        hipStream_t st = (hipStream_t)stream;
        CSE_HIP_TRY(hipMemcpyAsync(&n_fb, P.design.kind == CSE_HIER4 ? P.d_h4fb : P.d_b2fb, sizeof n_fb,
                                   hipMemcpyDeviceToHost, st));
        CSE_HIP_TRY(hipStreamSynchronize(st));
        out[0] = (int64_t)n_fb;
        out[1] = out[2] = out[3] = 0;
        return CSE_OK;
    }
    if (P.design.kind != CSE_PHASE23) {
        set_error("cse_work_counters: only the Phase II/III, 2-arm and 4-arm designs count their work");
        return CSE_EUNSUPPORTED;
    }
    unsigned long long h[4] = {0, 0, 0, 0};
    hipStream_t st = (hipStream_t)stream;
    CSE_HIP_TRY(hipMemcpyAsync(h, P.d_p23stats, sizeof h, hipMemcpyDeviceToHost, st));
    CSE_HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < 4; ++i) out[i] = (int64_t)h[i];
    return CSE_OK;
}

int cse_posterior_table(const cse_platten *p, float *out, int64_t capacity, int64_t *n_out,
                        void *stream) {
    if (int e = check_handle(p, "cse_posterior_table")) return e;
    const auto &P = p->P;
    if ((P.design.kind != CSE_HIER4 && P.design.kind != CSE_BASKET4) || !P.d_h4tbl) {
        set_error("cse_posterior_table: the platten's design has no posterior table");
        return CSE_EUNSUPPORTED;
    }
    if (!n_out) {
        set_error("cse_posterior_table: NULL n_out");
        return CSE_EINVAL;
    }
    *n_out = P.h4_outcomes;
    if (!out) return CSE_OK;
    if (capacity < 4 * P.h4_outcomes) {
        set_error("cse_posterior_table: capacity below 4 floats per outcome");
        return CSE_EINVAL;
    }
    CSE_HIP_TRY(hipMemcpyAsync(out, P.d_h4tbl, (size_t)P.h4_outcomes * 4 * sizeof(float),
                               hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return CSE_OK;
}

int cse_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
    return CSE_OK;
}

int cse_profile_get(const char *name, int64_t *launches, double *total_ms) {
    if (!name || !launches || !total_ms) {
        set_error("cse_profile_get: NULL argument");
        return CSE_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_prof_mu);
    prof_collect();
    auto it = g_totals.find(name);
    *launches = it == g_totals.end() ? 0 : it->second.first;
    *total_ms = it == g_totals.end() ? 0.0 : it->second.second;
    return CSE_OK;
}

int cse_profile_reset(void) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    prof_collect();
    g_totals.clear();
    return CSE_OK;
}

}  // extern "C"
