// adagrid.cpp -- adaptive gridding and simulation allocation from pilot runs (host).
//
// The paper reports its Phase II/III calibration on an adaptive grid: pilot simulations
// choose each tile's size and simulation count (Section 10.2).  One round of the library's
// rule: per box a decision from its tiles' results (done, split into 2^d children of half
// the half-width, double N, or stuck at the limits), then the new box list.  The GPU passes
// between rounds are the ordinary cse_validate / cse_calibrate calls on the boxes that
// changed.
#include <math.h>

#include <algorithm>
#include <limits>
#include <string>
#include <vector>

#include "cse_internal.h"

namespace {

constexpr int32_t DEC_DONE = 0, DEC_SPLIT = 1, DEC_DOUBLE = 2, DEC_STUCK = 3;

// split if `split_first` and allowed, else double if allowed, else split if allowed, else stuck
int32_t choose(bool split_first, bool can_split, bool can_double) {
    if (split_first && can_split) return DEC_SPLIT;
    if (can_double) return DEC_DOUBLE;
    if (can_split) return DEC_SPLIT;
    return DEC_STUCK;
}

}  // namespace

extern "C" {

int cse_adagrid_decide(const cse_adagrid_rule *rule, int64_t n_boxes, const double *radii, const int32_t *sims,
                       int64_t n_tiles, const int64_t *tile_box, const double *a, const double *b, const double *c,
                       int32_t *decision) {
    if (!rule || n_boxes < 0 || n_tiles < 0 || (n_boxes && (!radii || !sims || !decision)) ||
        (n_tiles && (!tile_box || !a || !b || !c))) {
        cse::set_error("cse_adagrid_decide: NULL argument or negative size");
        return CSE_EINVAL;
    }
    const int d = rule->d;
    if (d < 1 || d > 4 || (rule->mode != 0 && rule->mode != 1) || !(rule->r_min >= 0.0) || rule->n_max < 1) {
        cse::set_error("cse_adagrid_decide: bad rule (d in 1..4, mode 0 or 1, r_min >= 0, n_max >= 1)");
        return CSE_EINVAL;
    }
    for (int64_t t = 0; t < n_tiles; ++t)
        if (tile_box[t] < 0 || tile_box[t] >= n_boxes) {
            cse::set_error("cse_adagrid_decide: tile_box out of range");
            return CSE_EINVAL;
        }
    const double NaN = std::numeric_limits<double>::quiet_NaN();
    auto can_split = [&](int64_t i) {
        double m = INFINITY;
        for (int k = 0; k < d; ++k) m = std::min(m, radii[i * d + k]);
        return m / 2.0 >= rule->r_min;
    };
    auto can_double = [&](int64_t i) { return 2 * (int64_t)sims[i] <= rule->n_max; };
    std::fill(decision, decision + n_boxes, DEC_DONE);
    if (rule->mode == 0) {
        // validation: a = tile bound, b = cp_upper, c = R / N
        std::vector<double> U(n_boxes, NaN), G(n_boxes, NaN), M(n_boxes, NaN);
        auto upd = [](double &x, double v) { x = std::isnan(x) ? v : std::max(x, v); };
        for (int64_t t = 0; t < n_tiles; ++t) {
            const int64_t i = tile_box[t];
            upd(U[i], a[t]);
            upd(G[i], a[t] - b[t]);
            upd(M[i], b[t] - c[t]);
        }
        for (int64_t i = 0; i < n_boxes; ++i) {
            if (std::isnan(U[i]) || U[i] <= rule->target) continue;
            decision[i] = choose(G[i] >= M[i], can_split(i), can_double(i));
        }
        return CSE_OK;
    }
    // calibration: a = lambda, b = alpha', c = N
    double lam_star = INFINITY;
    for (int64_t t = 0; t < n_tiles; ++t) lam_star = std::min(lam_star, a[t]);
    std::vector<int64_t> best(n_boxes, -1);   // tile with the box's smallest lambda, first on ties
    for (int64_t t = 0; t < n_tiles; ++t) {
        const int64_t i = tile_box[t];
        if (best[i] < 0 || a[t] < a[best[i]]) best[i] = t;
    }
    double thr = lam_star + rule->margin;
    if (std::isnan(thr)) thr = INFINITY;   // lambda* = -inf with an infinite margin: every box
    for (int64_t i = 0; i < n_boxes; ++i) {
        const int64_t t = best[i];
        if (t < 0 || !(a[t] <= thr)) continue;
        const double ap = b[t];
        const double slack = rule->alpha - ap;
        const double spread = sqrt(std::max(ap * (1.0 - ap), 0.0) / (c[t] + 2.0));
        decision[i] = choose(slack >= spread, can_split(i), can_double(i));
    }
    return CSE_OK;
}

int cse_adagrid_apply(int32_t d, int64_t n_boxes, const double *theta, const double *radii, const int32_t *sims,
                      const int32_t *decision, int64_t cap, double *theta_out, double *radii_out,
                      int32_t *sims_out, int64_t *parent_out, int32_t *changed_out, int64_t *n_out) {
    if (d < 1 || d > 4 || n_boxes < 0 || !n_out || (n_boxes && (!theta || !radii || !sims || !decision))) {
        cse::set_error("cse_adagrid_apply: bad d, size or NULL argument");
        return CSE_EINVAL;
    }
    int64_t n = 0;
    for (int64_t i = 0; i < n_boxes; ++i) {
        if (decision[i] < DEC_DONE || decision[i] > DEC_STUCK) {
            cse::set_error("cse_adagrid_apply: decision codes are 0..3");
            return CSE_EINVAL;
        }
        if (decision[i] == DEC_DOUBLE && 2 * (int64_t)sims[i] > INT32_MAX) {
            cse::set_error("cse_adagrid_apply: doubled simulation count exceeds int32");
            return CSE_EINVAL;
        }
        n += decision[i] == DEC_SPLIT ? (int64_t)1 << d : 1;
    }
    *n_out = n;
    if (!theta_out) return CSE_OK;   // size query
    if (cap < n || !radii_out || !sims_out) {
        cse::set_error("cse_adagrid_apply: output capacity " + std::to_string(cap) + " < " + std::to_string(n) +
                       " or NULL output");
        return CSE_EINVAL;
    }
    int64_t j = 0;
    for (int64_t i = 0; i < n_boxes; ++i) {
        if (decision[i] == DEC_SPLIT) {
            // children c = 0 .. 2^d - 1: coordinate k in the upper half when bit k of c is set
            for (int64_t ch = 0; ch < ((int64_t)1 << d); ++ch, ++j) {
                for (int k = 0; k < d; ++k) {
                    const double r = radii[i * d + k] / 2.0;
                    theta_out[j * d + k] = theta[i * d + k] + (((ch >> k) & 1) ? r : -r);
                    radii_out[j * d + k] = r;
                }
                sims_out[j] = sims[i];
                if (parent_out) parent_out[j] = i;
                if (changed_out) changed_out[j] = 1;
            }
        } else {
            for (int k = 0; k < d; ++k) {
                theta_out[j * d + k] = theta[i * d + k];
                radii_out[j * d + k] = radii[i * d + k];
            }
            sims_out[j] = decision[i] == DEC_DOUBLE ? 2 * sims[i] : sims[i];
            if (parent_out) parent_out[j] = i;
            if (changed_out) changed_out[j] = decision[i] == DEC_DOUBLE ? 1 : 0;
            ++j;
        }
    }
    return CSE_OK;
}

}  // extern "C"
