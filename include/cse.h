/*
 * cse.h -- C ABI of the MI355X (gfx950) Continuous Simulation Extension library (libcse.so).
 *
 * Method: Yang, Thompson & Sklar, "Guarantees for Comprehensive Simulation
 * Assessment of Statistical Methods".  The library simulates a trial design at
 * the points of a platten (Section 5, Definition 1), counts rejections, forms
 * score-function gradient sums, selects the calibrated threshold of each tile
 * as an order statistic (Section 7.1), and evaluates the Clopper-Pearson plus
 * Tilt-Bound over each tile (Sections 6.1-6.2, 7.2).
 *
 * Conventions for every entry point:
 *   - Status: CSE_OK (0) or a negative cse_status; errors never cross the ABI
 *     as exceptions.  cse_last_error() returns a thread-local message for the
 *     last non-OK status of the calling thread.
 *   - Memory: arrays named "host" are read during the call only; all other
 *     array arguments are DEVICE pointers owned by the caller, written
 *     asynchronously on `stream` (a hipStream_t passed as void*, NULL = the
 *     null stream).  The library never frees caller memory.  Workspace the
 *     library needs is allocated at platten creation or on first use and
 *     released by cse_platten_destroy.
 *   - Calls are asynchronous: a CSE_OK status covers argument validation and
 *     launch errors; results are ready when `stream` is synchronised.
 *   - A "tile" below is one piece box ∩ P(b) of a caller box with non-empty
 *     interior (null configuration b, Section 5).  Tiles are numbered in box
 *     order, then by b ascending.  cse_platten_describe maps them back.
 *   - Random numbers: simulation k of every tile uses the words
 *     Philox4x32-10(key = (seed lo, seed hi), ctr = (w/4, k, 0, 0))[w mod 4]
 *     (Salmon et al., SC'11), i.e. common random numbers across tiles, which
 *     the calibration guarantee allows (Section 7.3).
 */
#ifndef CSE_H
#define CSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CSE_OK = 0,
    CSE_EINVAL = -1,       /* invalid argument (sizes, probabilities, pointers)   */
    CSE_ENOMEM = -2,       /* device or host allocation failed                    */
    CSE_EHIP = -3,         /* a HIP runtime call or a kernel launch failed        */
    CSE_EUNSUPPORTED = -4, /* design/option not supported                         */
    CSE_ECALIB = -5        /* calibration: every tile has k_i = 0 (Theorem 4 range) */
} cse_status;

/* Designs (the protocol D that maps simulated data to a rejection / statistic S). */
typedef enum {
    /* One-sided z-test (Section 4.2): X ~ N(theta, 1), H0: theta <= 0, reject X > cut;
     * calibration statistic S = -X.  d = 1. */
    CSE_ZTEST1 = 1,
    /* Two Bernoulli arms with n patients each (arm 0 control, arm 1 treatment, natural
     * parameter = logit), H0: theta1 <= theta0, pooled two-proportion z, reject z > cut;
     * calibration statistic S = -z.  d = 2. */
    CSE_BINOM2_Z = 2,
    /* Four Bernoulli arms, n patients each (arm 0 control), hierarchical model of
     * Section 10.1 (theta_i ~ N(mu, sigma^2), mu ~ N(-1.34, 100), sigma^2 ~ IG(0.0005,
     * 0.000005)); H_i: theta_i <= theta_0 for i = 1..3; statistic for null configuration
     * b: S_b = min_{i in b} (1 - P(p_i > p_0 | y)); reject when S_b < cut.  d = 4. */
    CSE_HIER4 = 3,
    /* Phase II/III Bayesian selection design (Section 10.2 and its appendix): four Bernoulli
     * arms (arm 0 control) embedded with n_per_arm = 350 potential patients each (Section 9);
     * Phase II of up to 400 patients with three looks (arm dropping for p_best < 0.15,
     * selection when p_success > 0.70, 0.60 at the last look), Phase III of up to 200 + 200
     * on the selected arm s and control with an interim (success when
     * P(p_s > p_0) > 0.95, futility when p_success < 0.20) and a final analysis that rejects
     * H_s when P(p_s > p_0) > 1 - cut.  Decisions use the hierarchical model of CSE_HIER4 with
     * the observed sample sizes.  Statistic for null configuration b: -inf for an early
     * success with s in b, 1 - P_final(p_s > p_0) for a final analysis with s in b, +inf
     * otherwise; a false rejection at lambda is S < lambda.  d = 4. */
    CSE_PHASE23 = 4,
    /* Bayesian basket trial (Section 10.1, the validation case study after Berry et al.):
     * four arms of n patients, arm a against its fixed rate p_0a (theta0[a] = logit p_0a),
     * hierarchical model of CSE_HIER4 on the offsets theta_a - theta0[a]; H_a: theta_a <=
     * theta0[a] for a = 0..3 (bit a of b); statistic S_b = min_{a in b} (1 - P(p_a > p_0a | y)),
     * reject when S_b < cut (0.15: the 85% rule).  The null boundaries are axis-aligned, so each
     * piece box ∩ P(b) is a box: boxes are cut at the boundaries they straddle and every piece
     * with b != 0 is a tile simulated at its own centre (cse_platten_tiles).  d = 4. */
    CSE_BASKET4 = 5
} cse_design_kind;

typedef struct {
    int32_t kind;       /* cse_design_kind                                      */
    int32_t n_arms;     /* d: 1 (ZTEST1), 2 (BINOM2_Z), 4 (HIER4, PHASE23, BASKET4) */
    int32_t n_per_arm;  /* patients per arm: 35 for BINOM2_Z, HIER4 and BASKET4, 350 (the
                           embedding) for PHASE23; ignored for ZTEST1             */
    int32_t reserved;   /* must be 0                                             */
    double cut;         /* fixed rule of the design used by cse_simulate/validate */
    double theta0[4];   /* BASKET4: logit of each arm's fixed rate p_0a; ignored otherwise */
} cse_design;

typedef struct cse_platten cse_platten;

/* Platten flags. */
#define CSE_PLATTEN_KEEP_ALL 1 /* single-hypothesis designs: keep boxes that meet no
                                  null (their tile is the whole box, in_null = 0)   */

/*
 * cse_platten_create -- build the platten of Definition 1 (Section 5) from caller boxes.
 *   design   host, read once.
 *   n_boxes  number of boxes (>= 1).
 *   theta    host, float64 [n_boxes][d], the simulation point of each box (its centre).
 *   radii    host, float64 [n_boxes][d], box half-widths (> 0).
 *   sims     host, int32 [n_boxes], simulations per box (1 .. 2^24).
 *   flags    0 or CSE_PLATTEN_KEEP_ALL.
 *   out      receives the handle (destroy with cse_platten_destroy).
 * Splits each box into tiles box ∩ P(b) with non-empty interior (eq. of the null
 * partition, Section 5), enumerates each tile's vertices in float64 (the supremum of
 * the bound over a convex polytope is attained at a vertex, Theorem 3), computes the
 * per-arm Bernoulli thresholds round(2^32 expit(theta)) in float64, plans the tile
 * batches the kernels run, and uploads everything to the current HIP device.
 * Errors: CSE_EINVAL (bad sizes/values, no box meets a null), CSE_ENOMEM, CSE_EHIP.
 */
int cse_platten_create(const cse_design *design, int64_t n_boxes, const double *theta,
                       const double *radii, const int32_t *sims, int32_t flags,
                       cse_platten **out);

/* Release the platten and its device workspaces (synchronises the device first). */
int cse_platten_destroy(cse_platten *p);

/* Number of tiles (box pieces) in the platten; < 0 on a NULL handle. */
int64_t cse_platten_size(const cse_platten *p);

/*
 * cse_platten_tiles -- host copies of each tile's simulation point and half-widths
 * (float64 [n_tiles][d] each, either may be NULL): the box's centre and half-widths, except
 * for CSE_BASKET4, whose tiles are the pieces of a box cut at the null boundaries.
 * Errors: CSE_EINVAL (NULL platten).
 */
int cse_platten_tiles(const cse_platten *p, double *theta, double *radii);

/*
 * cse_platten_describe -- host copies of the tile list (any pointer may be NULL):
 *   box      int64 [n_tiles]  box index of each tile
 *   cfg      int32 [n_tiles]  null configuration b (bit j-1 = hypothesis j is true)
 *   n_vert   int32 [n_tiles]  number of vertices of box ∩ P(b)
 *   in_null  int32 [n_tiles]  1 when the tile lies in the null space
 */
int cse_platten_describe(const cse_platten *p, int64_t *box, int32_t *cfg, int32_t *n_vert,
                         int32_t *in_null);

/*
 * cse_simulate -- Monte Carlo at every tile with the design's fixed rule (Section 6.1 input).
 *   reject   int32 [n_tiles]       R_i = number of simulations whose F_b(X) = 1 (FWER event of
 *                                  the tile's configuration b, Section 5).
 *   score_T  int64 [n_tiles][d] or NULL: binomial designs, sum over rejecting simulations of
 *                                  the sufficient statistic T(x) (arm success counts, Example 1);
 *                                  PHASE23: int64 [n_tiles][2d], the sums of the observed success
 *                                  counts y_a, then of the observed sample sizes n_a.
 *   score_Z  float64 [n_tiles] or NULL: ZTEST1, sum over rejecting simulations of X - theta.
 *   grad     float64 [n_tiles][d] or NULL: score-function estimate of d f / d theta,
 *                                  (sum_rej T(x) - R grad A(theta)) / N  (exponential family);
 *                                  PHASE23: (sum_rej y_a - sum_rej n_a expit(theta_a)) / N (the
 *                                  unobserved embedded patients contribute zero in expectation).
 *                                  HIER4 and BASKET4 give score_T [n_tiles][4] (arm success
 *                                  counts summed over the simulations whose event at the tile's
 *                                  configuration b holds) and grad as for the binomial designs;
 *                                  score_Z is ZTEST1 only (CSE_EUNSUPPORTED otherwise).
 * Errors: CSE_EINVAL (NULL reject, bad handle), CSE_EHIP.
 */
int cse_simulate(const cse_platten *p, uint64_t seed, int32_t *reject, int64_t *score_T,
                 double *score_Z, double *grad, void *stream);

/*
 * cse_validate -- Validation procedure (Algorithm 1, Section 6): simulate as cse_simulate, then
 *   cp_upper   float64 [n_tiles] Clopper-Pearson (1-delta) upper bound at theta_i (Section 6.1)
 *   tile_bound float64 [n_tiles] inf_q max_{v in vertices} U(theta_i, v, q, cp_upper_i)
 *                                (Tilewise Optimized Tilt-Bound, Remark 3, Section 6.2)
 *   q_star     float64 [n_tiles] or NULL: the optimising Holder exponent q.
 * reject/score_T/score_Z/grad as in cse_simulate (score pointers may be NULL).
 * Errors: CSE_EINVAL (delta outside (0,1)), CSE_EHIP.
 */
int cse_validate(const cse_platten *p, uint64_t seed, double delta, int32_t *reject,
                 int64_t *score_T, double *score_Z, double *grad, double *cp_upper,
                 double *tile_bound, double *q_star, void *stream);

/*
 * cse_calibrate -- Calibration procedure (Algorithm 2, Section 7):
 *   alpha_prime   float64 [n_tiles]  sup_q min_v U^{-1}(theta_i, v, q, alpha) (Section 7.2)
 *   k             int32   [n_tiles]  floor((N_i + 1) alpha'_i)
 *   lambda_tile   float64 [n_tiles]  lambda*_i = S_(k_i), the k_i-th smallest statistic of the
 *                                    tile (Section 7.1); -inf when k_i = 0
 *   lambda_global float64 [1]        min of lambda*_i over the tiles in the null space (Section
 *                                    7.3; with CSE_PLATTEN_KEEP_ALL the tiles outside it are
 *                                    simulated and selected but do not bound lambda*)
 *   reject_at_lambda int32 [n_tiles] or NULL: #{simulations with S < lambda*_i}
 * Validation outputs at the design's fixed rule (reject, score_T, score_Z, grad, cp_upper,
 * tile_bound) may be requested in the same pass (each may be NULL; cp_upper/tile_bound use
 * `delta`, which is ignored when both are NULL).
 * Errors: CSE_EINVAL (alpha or delta outside (0,1)), CSE_ENOMEM (key workspace), CSE_EHIP.
 * Tiles with k_i = 0 get lambda*_i = -inf (no calibrated rejection); CSE_ECALIB is not
 * raised from the asynchronous path -- check lambda_global on the host.
 */
int cse_calibrate(const cse_platten *p, uint64_t seed, double alpha, double *alpha_prime,
                  int32_t *k, double *lambda_tile, double *lambda_global,
                  int32_t *reject_at_lambda, double delta, int32_t *reject, int64_t *score_T,
                  double *score_Z, double *grad, double *cp_upper, double *tile_bound,
                  void *stream);

/*
 * cse_calibrate_noalloc -- cse_calibrate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).  Same arguments,
 * launches and results as cse_calibrate, but the calibration keys live in a static workspace of
 * CSE_NOALLOC_SCRATCH_BYTES bytes compiled into the library (one copy per device, resident until the
 * process ends) instead of memory allocated on the first calibration: the call allocates and frees
 * nothing.  The keys need 16 bytes per key slot for CSE_BINOM2_Z (one record of success counts per
 * simulation and tile batch) or 4 bytes for the other designs (one float32 statistic per simulation
 * and tile), n_key_slots of cse_platten_stats; a larger platten is refused with CSE_EINVAL.
 * Every call on a device shares that device's workspace, which keeps the last call's contents:
 * calls whose execution overlaps on one device (other streams or threads) race and must be
 * ordered by the caller, as calls on one platten must be anyway.  The first call on a device looks
 * the workspace's address up (hipGetSymbolAddress) with that device current.
 * Errors: as cse_calibrate, plus CSE_EINVAL (keys exceed the workspace) and CSE_EHIP (lookup failed).
 */
#define CSE_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
int cse_calibrate_noalloc(const cse_platten *p, uint64_t seed, double alpha, double *alpha_prime,
                          int32_t *k, double *lambda_tile, double *lambda_global,
                          int32_t *reject_at_lambda, double delta, int32_t *reject, int64_t *score_T,
                          double *score_Z, double *grad, double *cp_upper, double *tile_bound,
                          void *stream);

/*
 * cse_bound -- the float64 bound of each tile, without simulation.
 *   mode 0 (validate): R int32 [n_tiles] device rejection counts; out = tilewise optimized
 *          Tilt-Bound of the Clopper-Pearson bound at level delta_or_alpha = delta.
 *   mode 1 (invert):   R ignored (may be NULL); out = alpha' for level delta_or_alpha = alpha.
 *   mode 2 (tilt only): R ignored; `a` float64 [n_tiles] device values f(theta_i) in [0,1];
 *          out = inf_q max_v U(theta_i, v, q, a_i) (Remark 3).
 *   q_star float64 [n_tiles] or NULL.
 * The optimisation over q (s = log(q - 1) in [-30, 30], quasi-convex by Theorem 2) is a parallel
 * section search with eight lanes per tile (12 rounds of 8 points) on plattens below 2^18 tiles
 * and Brent's search (parabolic and golden-section steps) with one lane per tile from 2^18 tiles on; each
 * returns the best point it evaluated, and the two agree within 1e-9 relative on the same tile.
 * Errors: CSE_EINVAL, CSE_EHIP.
 */
int cse_bound(const cse_platten *p, int32_t mode, const int32_t *R, const double *a,
              double delta_or_alpha, double *out, double *q_star, void *stream);

/*
 * cse_taylor -- the second-order Taylor comparison bound of Section 4.3 over each tile, and the
 * gradient-guided worst-case candidate point of the tile.
 *   f      float64 [n_tiles]    f(theta_i) to expand from (the exact value for a comparison,
 *                               or an upper confidence bound such as cp_upper in practice)
 *   grad   float64 [n_tiles][d] the gradient at theta_i (exact, or the score estimate of
 *                               cse_simulate / cse_validate)
 *   bound  float64 [n_tiles]    max over the tile's vertices v of
 *                               f + grad.v + (1/2) sum_a h_a v_a^2, clipped to 1, where h_a is
 *                               the supremum over the tile's box of d^2 A / d theta_a^2 (1 for
 *                               the z-test, n p (1 - p) for a binomial arm), which bounds the
 *                               remainder of a rejection probability in the exponential family
 *                               (the paper's f'' <= 1 for the z-test)
 *   vertex int32 [n_tiles] or NULL: index of the maximising vertex (first on ties; vertex order
 *                               as in cse_platten_describe's enumeration)
 *   point  float64 [n_tiles][d] or NULL: that vertex, theta_i + v (the worst-case candidate)
 * The bound is convex in v, so its maximum over the convex tile is attained at a vertex.
 * Errors: CSE_EINVAL (NULL f, grad or bound), CSE_EHIP.
 */
int cse_taylor(const cse_platten *p, const double *f, const double *grad, double *bound, int32_t *vertex,
               double *point, void *stream);

/*
 * cse_validate_lower -- the lower side of a two-sided validation band (Remark 2, Section 4.1: the
 * Tilt-Bound applied to 1 - F gives f(theta0 + v) >= 1 - U(theta0, v, q, 1 - f(theta0))).
 *   R        int32 [n_tiles] device rejection counts of this platten's tiles (the `reject`
 *                            output of cse_simulate / cse_validate / cse_calibrate)
 *   cp_lower float64 [n_tiles] or NULL: Clopper-Pearson (1-delta) lower bound
 *                            Beta^{-1}(delta; R, N - R + 1) at theta_i (0 when R = 0), computed
 *                            as 1 - cp_upper(N - R) (Section 6.1)
 *   lower    float64 [n_tiles] 1 - inf_q max_v U(theta_i, v, q, 1 - cp_lower_i): with
 *                            probability >= 1 - delta, f >= lower on the whole tile
 *                            (with cse_validate's tile_bound: a band at level 1 - 2 delta)
 *   q_star   float64 [n_tiles] or NULL: the optimising Holder exponent.
 * Errors: CSE_EINVAL (NULL R or lower, delta outside (0,1)), CSE_EHIP.
 */
int cse_validate_lower(const cse_platten *p, const int32_t *R, double delta, double *cp_lower, double *lower,
                       double *q_star, void *stream);

/*
 * cse_confidence_set -- confidence set from a calibration (Section 8).  Each tile's test
 * rejects the observed statistic when s_i < lambda_i; the confidence region is the union of
 * the tiles it does not reject, and the confidence set of an estimand e(theta) is the image of
 * that region.
 *   s_obs       float64 device, the observed statistic: [n_tiles] (s_stride 1) or one value
 *               for every tile (s_stride 0).  Compared in the precision of the design's
 *               simulated statistic: float64 for CSE_BINOM2_Z, float32 otherwise.
 *   lambda_tile float64 [n_tiles] device, the tiles' calibrated thresholds (cse_calibrate's
 *               lambda_tile at the chosen alpha; -inf keeps a tile whatever s is)
 *   coef        float64 [d + 1] HOST: e(theta) = coef[d] + sum_a coef[a] g(theta_a)
 *   link        0: g = identity (range over the tile = min / max over its vertices, exact);
 *               1: g = expit, e.g. p_1 - p_0 (each term's extremes over the tile's bounding
 *               box: exact on a box, an enclosing interval on a clipped tile)
 *   keep        int32 [n_tiles]   1 when the tile is in the confidence region
 *   e_lo, e_hi  float64 [n_tiles] range of e over each tile (kept or not)
 *   e_range     float64 [2] device: (min e_lo, max e_hi) over kept tiles; (+inf, -inf) when
 *               no tile is kept.
 * Coverage is that of the calibration (>= 1 - alpha); for a two-sided interval intersect an
 * upper and a lower one, each at level alpha / 2.
 * Errors: CSE_EINVAL (NULL pointers, link or s_stride out of range, non-finite coef), CSE_EHIP.
 */
int cse_confidence_set(const cse_platten *p, const double *s_obs, int64_t s_stride, const double *lambda_tile,
                       const double *coef, int32_t link, int32_t *keep, double *e_lo, double *e_hi,
                       double *e_range, void *stream);

/*
 * cse_calibrate_tiebreak -- randomised calibration (the adjoined uniform discussed with
 * Theorem (pointwise calibration), Section 7.1): every simulation k also draws
 * u_k = first word of Philox4x32-10(key = seed, counter = (0, k, 1, 0)) (shared by all tiles,
 * disjoint from the data words), the statistic is the pair (S, u) and the threshold the pair
 * (lambda, c), both ordered lexicographically; a new observation (s, u) is rejected when
 * s < lambda, or s == lambda and u < c.  This removes the discreteness term of the
 * calibration's mean and variance.
 *   alpha_prime, k  as cse_calibrate (k may be NULL, alpha_prime may be NULL)
 *   lambda_tile     float64 [n_tiles], u_tile uint32 [n_tiles]: the k_i-th smallest pair
 *                   ((-inf, 0) when k_i = 0)
 *   lambda_global   float64 [1], u_global uint32 [1]: the lexicographic minimum over the
 *                   tiles in the null space
 *   reject_at_lambda int32 [n_tiles]: pairs strictly below (lambda_i, c_i) (k_i - 1 when the
 *                   tied simulations' u are distinct)
 * Errors: CSE_EINVAL (alpha outside (0,1), NULL outputs, empty platten), CSE_ENOMEM, CSE_EHIP.
 */
int cse_calibrate_tiebreak(const cse_platten *p, uint64_t seed, double alpha, double *alpha_prime, int32_t *k,
                           double *lambda_tile, uint32_t *u_tile, double *lambda_global, uint32_t *u_global,
                           int32_t *reject_at_lambda, void *stream);

/*
 * Adaptive gridding and simulation allocation from pilot runs (the paper's Phase II/III
 * calibration chooses tile sizes and simulation counts adaptively, Section 10.2).  Host-only
 * calls: all arrays are HOST memory; no GPU work.  One round of the rule, between the GPU
 * passes (cse_validate or cse_calibrate on the boxes that changed):
 *
 * cse_adagrid_decide -- per-box decision from its tiles' results:
 *   rule->mode 0 (validation): a = tile_bound, b = cp_upper, c = R / N per tile.  A box whose
 *     largest bound U <= target is done (0).  Otherwise: G = max(bound - cp_upper) (the
 *     part a smaller tile removes), M = max(cp_upper - R/N) (the part more simulations
 *     remove); split (1) when G >= M, else double N (2).
 *   rule->mode 1 (calibration): a = lambda_i, b = alpha'_i, c = N_i per tile; lambda* = min
 *     over the tiles given.  A box is critical when its smallest lambda_i <= lambda* + margin
 *     (every box when margin = +inf);
 *     for that tile, split when alpha - alpha'_i >= sqrt(alpha'(1 - alpha')/(N + 2)) (the
 *     spread of f(lambda_hat) ~ Beta(k, N - k + 1), Theorem 4), else double N.
 *   Either way a split needs min half-width / 2 >= r_min and doubling needs 2 N <= n_max;
 *   when the preferred move is not allowed the other one is taken, and a box that can do
 *   neither is stuck (3).  Boxes without tiles are done.
 *   radii [n_boxes][d], sims [n_boxes], tile_box [n_tiles] (box index of each tile),
 *   decision int32 [n_boxes] out.
 * cse_adagrid_apply -- the next box list: a split box is replaced in place by its 2^d
 *   children (child c has coordinate k in the upper half when bit k of c is set, half-width
 *   r/2, the parent's N); a doubled box keeps its place with 2 N; others are copied.
 *   With theta_out == NULL only *n_out (the new count) is written.  parent_out [n_out] (or
 *   NULL): index of the box each new box comes from; changed_out [n_out] (or NULL): 1 for
 *   children and doubled boxes (the ones to simulate next).
 * Errors: CSE_EINVAL (bad rule, sizes, codes, capacity, or an N that would exceed int32).
 */
typedef struct cse_adagrid_rule {
    int32_t mode;    /* 0 validation, 1 calibration */
    int32_t d;       /* parameter dimension (1..4) */
    double target;   /* validation: largest acceptable tile bound */
    double alpha;    /* calibration: the level */
    double margin;   /* calibration: critical boxes have lambda <= lambda* + margin */
    double r_min;    /* smallest half-width a split may produce */
    int64_t n_max;   /* largest simulation count a doubling may produce */
} cse_adagrid_rule;

int cse_adagrid_decide(const cse_adagrid_rule *rule, int64_t n_boxes, const double *radii, const int32_t *sims,
                       int64_t n_tiles, const int64_t *tile_box, const double *a, const double *b, const double *c,
                       int32_t *decision);
int cse_adagrid_apply(int32_t d, int64_t n_boxes, const double *theta, const double *radii, const int32_t *sims,
                      const int32_t *decision, int64_t cap, double *theta_out, double *radii_out,
                      int32_t *sims_out, int64_t *parent_out, int32_t *changed_out, int64_t *n_out);

/*
 * Plans: one validation or calibration step captured once into a HIP graph and replayed.
 * The step is exactly the launches of cse_validate / cse_calibrate with the same arguments
 * (Algorithms 1 and 2: alpha' -> simulation -> selection -> reductions -> bound); every
 * pointer, the seed and the levels are fixed when the plan is made, so each replay writes
 * the same outputs as the eager call would.  The calibration key workspace is allocated
 * before capture; the graph contains kernel launches only.
 *   cse_plan_validate / cse_plan_calibrate: arguments and errors as cse_validate /
 *        cse_calibrate (no stream: capture uses a private stream); out receives the plan.
 *   cse_plan_launch: enqueue one replay on `stream` (asynchronous).  Replays of one plan,
 *        and plans or eager calls on the same platten, share the platten's workspaces:
 *        order them on one stream.  A plan is tied to its platten's launch shape: after
 *        cse_autotune has rebuilt it, or after the platten is destroyed, cse_plan_launch returns
 *        CSE_EINVAL without replaying (capture a new plan; a plan must not be replayed after its
 *        platten is gone, and only cse_plan_destroy may be called on it then).
 *   cse_plan_nodes: number of graph nodes (-1 for NULL).
 *   cse_plan_destroy: synchronises the device and releases the graph; NULL is a no-op.
 * Errors: CSE_EINVAL, CSE_ENOMEM, CSE_EHIP (capture or instantiation failed).
 */
typedef struct cse_plan cse_plan;
int cse_plan_validate(const cse_platten *p, uint64_t seed, double delta, int32_t *reject,
                      int64_t *score_T, double *score_Z, double *grad, double *cp_upper,
                      double *tile_bound, double *q_star, cse_plan **out);
int cse_plan_calibrate(const cse_platten *p, uint64_t seed, double alpha, double *alpha_prime,
                       int32_t *k, double *lambda_tile, double *lambda_global,
                       int32_t *reject_at_lambda, double delta, int32_t *reject,
                       int64_t *score_T, double *score_Z, double *grad, double *cp_upper,
                       double *tile_bound, cse_plan **out);
int cse_plan_launch(const cse_plan *plan, void *stream);
int64_t cse_plan_nodes(const cse_plan *plan);
int cse_plan_destroy(cse_plan *plan);

/*
 * cse_autotune -- choose the launch shape of the platten's fused simulation kernel by timing
 * candidates on the current device (synchronises `stream`):
 *   CSE_ZTEST1:            waves of the grid, from {4096 .. 262144} (powers of 2);
 *   CSE_BINOM2_Z, HIER4, BASKET4: workgroups of the grid (simulation ranges per group of
 *                          batches), from {1024 .. 65536} (powers of 2; at least 4
 *                          chunks of 64 simulations per item), timed on the calibration
 *                          launch plus the validation launch;
 *   CSE_PHASE23:           trials per queue item {64, 128, 256, 512} x persistent grid
 *                          {512, 1024, 2048} workgroups, timed on a strided sample of tiles
 *                          holding at most max_trials trials.
 * The fastest is kept in the platten.  Results of every later call are unchanged (integer
 * reductions are order-independent and keys are laid out by tile, not by launch shape).
 * Plans captured on this platten before the call become stale (cse_plan_launch refuses them).
 *   out  host int64 [2]: the chosen value and, for CSE_PHASE23, the grid (else 0).
 * Errors: CSE_EINVAL (NULL out, max_trials < 1), CSE_ENOMEM, CSE_EHIP.
 */
int cse_autotune(cse_platten *p, uint64_t seed, int64_t max_trials, int64_t out[2], void *stream);

/*
 * cse_simulate_per_tile -- the plain forward-only path: one kernel launch per tile, no
 * common-random-number batching across tiles, rejection counts only (the design's fixed rule).
 * Same Philox stream and draw rules as cse_simulate, hence identical R.  Processes tiles
 * [tile_begin, tile_end).  Used as the reference point for the batched path's speed.
 * Errors: CSE_EINVAL, CSE_EHIP.
 */
int cse_simulate_per_tile(const cse_platten *p, uint64_t seed, int64_t tile_begin,
                          int64_t tile_end, int32_t *reject, void *stream);

/*
 * cse_work_counters -- work done by the last simulation launch on a CSE_PHASE23 platten
 * (cse_simulate / cse_validate / cse_calibrate): out (host int64 [4]) = trials simulated,
 * posterior evaluations at Phase II looks and at Phase III looks (the first look of every
 * trial is a table lookup and is not counted), Newton steps over all nodes of those looks.
 * On a CSE_BINOM2_Z platten: out[0] = tiles that the last calibration's bracketed selection
 * left to the exact full-histogram pass (k-th statistic outside the bracket, or the batch's
 * brackets too wide for the histogram), out[1..3] = 0.  On a CSE_HIER4 platten: out[0] = tiles
 * whose k-th key the last bracketed calibration did not hold among its candidates (selected
 * exactly from keys regenerated by the counter-based generator), out[1..3] = 0.
 * Synchronises `stream`.  Used to state the kernel's arithmetic per launch.
 * Errors: CSE_EINVAL (NULL out), CSE_EUNSUPPORTED (other designs), CSE_EHIP.
 */
int cse_work_counters(const cse_platten *p, int64_t out[4], void *stream);

/*
 * cse_platten_set_option -- tuning options of a platten (host call, no kernel launch).
 *   CSE_OPT_B2_MARGIN (CSE_BINOM2_Z calibration): the selection's bracket around each tile's
 *        k-th statistic, in standard deviations of the count (default 5).  Results do not
 *        depend on it: tiles whose k-th statistic falls outside the bracket take an exact
 *        full-histogram pass (cse_work_counters counts them); a smaller margin lists fewer
 *        simulations in the bracketed pass but sends more tiles to the exact one.  A plan
 *        captured earlier keeps the margin it was captured with.
 *   CSE_OPT_H4_BRACKET (CSE_HIER4 calibration): 1 selects from bracketed keys: a pilot pass keeps
 *        the float32 keys of the first 2,048 simulations, whose order statistics around rank
 *        (k/N) 2048 bracket each tile's k-th key; the fused pass over the other simulations
 *        counts the keys below the bracket and keeps only those inside it (about a tenth of the
 *        HBM traffic of storing every key).  0 (default) stores every float32 key and selects
 *        from them, as cse_calibrate_tiebreak always does.  Same results either way.  Turning
 *        it on allocates the candidate regions (device memory; about 20 KB per tile at 32,768
 *        simulations per tile with the default launch shape), turning it off frees them; the
 *        plattens whose batches hold more than 128 key rows keep the every-key path.
 *   CSE_OPT_H4_MARGIN (CSE_HIER4 bracketed calibration): the bracket's margin in standard
 *        deviations of the pilot rank (default 6, lowered towards 3 where the bracket would
 *        hold too many keys).  Results do not depend on it: a tile whose k-th key is not among
 *        the kept ones is selected from its keys regenerated one by one from the counter-based
 *        generator (slow; cse_work_counters counts them).
 * Errors: CSE_EINVAL (bad handle, unknown option, value outside [0, 100]; 0 or 1 for
 * CSE_OPT_H4_BRACKET), CSE_ENOMEM (the candidate regions could not be allocated).
 */
#define CSE_OPT_B2_MARGIN 1
#define CSE_OPT_H4_MARGIN 2
#define CSE_OPT_H4_BRACKET 3
int cse_platten_set_option(cse_platten *p, int32_t option, double value);

/*
 * cse_posterior_table -- the design table of a CSE_HIER4 platten: for every outcome
 * y in {0..n}^4 (index ((y0 (n+1) + y1) (n+1) + y2) (n+1) + y3) the float32 values
 * (1 - P(p_1 > p_0 | y), 1 - P(p_2 > p_0 | y), 1 - P(p_3 > p_0 | y), 0) of the hierarchical
 * model of Section 10.1 (posterior by 90-node quadrature over sigma^2, computed in float64
 * when the platten is created).
 *   out       device float32 [capacity] (4 floats per outcome), written on `stream`; may be NULL
 *   n_out     host, receives the number of outcomes ((n+1)^4)
 * Errors: CSE_EINVAL (NULL n_out, capacity too small), CSE_EUNSUPPORTED (other designs).
 */
int cse_posterior_table(const cse_platten *p, float *out, int64_t capacity, int64_t *n_out,
                        void *stream);

/*
 * cse_platten_stats -- sizes of the planned launch (host), out[0..11] =
 *   n_tiles, n_batches (tile batches of the fused kernel), n_work_items (waves or workgroups
 *   launched by one simulation pass), n_key_slots (calibration keys: CSE_BINOM2_Z one 16-byte record
 *   per (simulation, batch), other designs one float32 per (simulation, tile)), total simulations (sum of N
 *   over tiles), tiles per batch, max N, batch-simulation pairs (sum over batches of their N),
 *   workgroup-simulation pairs (sum over workgroup items of their simulation count; the unit of
 *   shared random-number generation), number of distinct N, microseconds spent building the
 *   design table at creation (CSE_HIER4 posterior table, CSE_PHASE23 first-look table, else
 *   0), the launch shape (CSE_ZTEST1 waves, CSE_BINOM2_Z / CSE_HIER4 workgroups, CSE_PHASE23
 *   trials per queue item; see cse_autotune).
 */
int cse_platten_stats(const cse_platten *p, int64_t out[12]);

/*
 * Kernel timing for measurement (process-wide, not thread-safe against concurrent calls):
 * while enabled, every kernel launch of the library is bracketed by two HIP events recorded
 * on the launch's own stream.  cse_profile_get synchronises the recorded events and returns,
 * for the kernel `name` (e.g. "binom2_calib"), the number of timed launches and their total
 * duration in milliseconds.  Do not enable while capturing a HIP graph.
 */
int cse_profile_enable(int32_t on);
int cse_profile_get(const char *name, int64_t *launches, double *total_ms);
int cse_profile_reset(void);

/* Thread-local message for the last non-OK status returned on this thread. */
const char *cse_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CSE_H */
