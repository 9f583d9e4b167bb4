// cse_internal.h -- data structures shared by the files of libcse.so (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <memory>
#include <string>
#include <vector>

#include "cse.h"

namespace cse {

constexpr int WAVE = 64;
constexpr int WG = 256;              // 4 waves per workgroup
constexpr int MAX_D = 4;
constexpr int NP35 = 35;             // patients per arm of the binomial designs
constexpr int P23_NMAX_ARM = 350;    // embedded patients per arm of the Phase II/III design
constexpr uint64_t PLATTEN_GONE = ~0ull;   // shape generation of a destroyed platten
constexpr int MIN_PARTS = 256;            // partial minima of the large min reductions

// ---- tile batches ("blocks"): each wave owns one block for a range of simulations ----
// 2-arm designs: an 8 x 8 product of distinct arm-0 and arm-1 thresholds, so one
// simulation's success counts at 16 thresholds serve 64 tiles (common random numbers).
constexpr int B2U = 8, B2V = 8;
struct Blk2 {
    uint32_t T0[B2U];          // arm-0 Bernoulli thresholds (uint32, see platten.cpp)
    uint32_t T1[B2V];          // arm-1 thresholds
    int32_t tile[B2U * B2V];   // tile id of slot (u, v) = u * B2V + v, or -1
    int32_t n_sims;            // simulations of every tile of this block
    int32_t pad;
    int64_t key_base;          // calibration records: simulation k of this block has its record
                               // (Rec2) at key_base + k (k < n_sims rounded up to 64)
};
// Calibration record of one simulation of a 2-arm block: the success counts at the block's
// thresholds, y0[u] in byte u of (w0, w1) and y1[v] in byte v of (w2, w3).  Every tile's outcome
// y0[u] (n+1) + y1[v] follows from it, so 16 bytes serve the block's 64 tiles.
constexpr int REC2_BYTES = 16;

// z-test: 64 tiles share each simulation's normal draw.
constexpr int B1T = 64;
struct Blk1 {
    float theta[B1T];
    int32_t tile[B1T];
    int32_t n_sims;
    int32_t pad;
    int64_t key_base;          // keys of slot s live at key_base + s * n_sims + k
};

// 4-arm designs: a 4 x 4 x 2 x 2 product of distinct thresholds (arms 0..3) = 64 box slots;
// slot (u0,u1,u2,u3) = ((u0 * 4 + u1) * 2 + u2) * 2 + u3.  A box's tiles (one per null
// configuration b present, b ascending) are consecutive key rows starting at row0[slot] and
// consecutive tile ids starting at tile0[slot]; bmask bit b marks configuration b.
constexpr int B4N0 = 4, B4N1 = 4, B4N2 = 2, B4N3 = 2;
constexpr int B4S = B4N0 * B4N1 * B4N2 * B4N3;
struct Blk4 {
    uint32_t T0[B4N0], T1[B4N1], T2[B4N2], T3[B4N3];
    int32_t row0[B4S];         // first key row of the slot's tiles, -1 when the slot has no box
    int32_t tile0[B4S];        // first tile id of the slot's box
    uint32_t bmask[B4S];       // configurations present (bit b, b = 1..7)
    int32_t n_rows;            // key rows (tiles) of this block
    int32_t n_sims;
    int64_t key_base;          // key of row r, simulation k at key_base + ((k/64) * n_rows + r) * 64 + k%64
};

// Work item: one wave simulates sims [k_begin, k_end) of block blk.
struct WorkItem {
    int32_t blk;
    uint32_t k_begin;
    uint32_t k_end;
    int32_t pad;
};

// Workgroup item of the 4-arm kernels: its 4 waves simulate the same sims [k_begin, k_end) for up
// to 4 blocks of equal N (blk = -1: no block), sharing each simulation's Philox words.
struct GroupItem {
    int32_t blk[4];
    uint32_t k_begin;
    uint32_t k_end;
    int32_t slice;   // index of the item's simulation range among its group's ranges
    int32_t pad;
};

// 4-arm calibration with bracketed keys: a pilot pass stores the keys of the first H4_PILOT
// simulations; per tile they give a bracket [lo, hi] around the k-th smallest key; the fused pass
// over the remaining simulations counts the keys below lo and keeps those in [lo, hi] in the
// tile's candidate regions (H4_PCAP slots for the pilot's, then h4_caps per item range).
constexpr int H4_PILOT = 2048;
constexpr int H4_PCAP = 1024;
constexpr int H4_MAXS = 1024;   // item ranges per group at most (the selection's region table)
constexpr int H4_BROWS = 128;   // key rows per wave whose counters live in LDS (the rest: global atomics)

// Workgroup item of the 2-arm kernel: its 16 waves simulate [k_begin, k_end) for the batches of a
// 4 x 4 square of the threshold grid (equal N): blk[4 r + c] is the batch of row group r (8 arm-0
// thresholds) and column group c (8 arm-1 thresholds) of the square (-1: none), so the square's
// 32 + 32 distinct thresholds serve 1,024 tiles.
constexpr int SQ2 = 4;                   // square side (batches)
constexpr int SQ2W = SQ2 * SQ2;          // waves per workgroup
struct SquareItem {
    int32_t blk[SQ2W];
    uint32_t k_begin;
    uint32_t k_end;
};

// Per-node constants of the hierarchical posterior (90 nodes equally spaced in log s2 on
// [log 1e-6, log 1e3]), computed once on the host: log s2, s2, 1/s2, c = 100 / (s2 + 400),
// beta = c / s2, and lconst = log|Q|/2 + log of the inverse-gamma density of s2 + log of the
// trapezoid weight in log s2 times s2.
constexpr int HIER_NODES = 90;
struct HierNode {
    double ls2, s2, inv_s2, c, beta, lconst;
};

// Arguments of the Phase II/III kernel (device pointers owned by the platten, except the
// outputs filled in per launch).
struct P23Args {
    const WorkItem *items;          // (tile in blk, simulation range) queue entries
    int64_t n_items;
    uint32_t *counter;              // queue head, zeroed before each launch
    const uint32_t *tileT;          // [n_tiles][4] Bernoulli thresholds
    const int32_t *cfg;             // [n_tiles] null configuration b
    const int64_t *key_off;         // [n_tiles] first key of the tile (keys contiguous per tile)
    uint32_t key0, key1;            // Philox key (seed)
    float cut;                      // lambda of the final analysis (the design's fixed rule)
    int32_t pad;
    uint32_t *R;                    // [n_tiles] rejections at cut
    unsigned long long *sumT;       // [n_tiles][8] sums of observed y_a, then n_a, over rejections
    float *keys;                    // calibration keys S or NULL
    unsigned long long *stats;      // NULL or [4]: trials, Phase II / Phase III posterior looks, Newton steps
    const double *gh;               // Gauss-Hermite rule (weight e^{-x^2}): nodes [16], weights [16]
    const HierNode *nodes;          // per-node constants of the hierarchical posterior [90]
    const uint8_t *look1;           // decision code of the first look per outcome, 51^4 entries
    double sqrt_pi, z95;            // sqrt(pi), Phi^{-1}(0.95)
};

// Family of the data model for the bound (Example 1 / Section 4.2).
enum Family : int32_t { FAM_NORMAL = 1, FAM_BINOM = 2 };

struct Platten {
    cse_design design{};
    int d = 0;              // parameter dimension
    int p = 0;              // number of null hypotheses
    int32_t family = 0;
    int32_t n_per_arm = 0;
    int64_t n_boxes = 0, n_tiles = 0;
    int device = 0;

    // host copies
    std::vector<int64_t> tile_box;
    std::vector<int32_t> tile_cfg, tile_nv, tile_in_null, tile_N;
    std::vector<double> tile_theta;      // [n_tiles * d]
    std::vector<int32_t> vert_off;       // [n_tiles + 1]
    std::vector<double> verts;           // [total vertices * d] displacements from theta
    std::vector<double> tile_radii;      // [n_tiles * d]
    std::vector<int32_t> tile_is_box;    // [n_tiles]
    int32_t max_N = 0;
    int64_t total_sims = 0;              // sum of N over tiles
    int64_t block_sims = 0;              // sum over batches of their N
    int64_t group_sims = 0;              // sum over workgroup items of their simulation count

    // device copies (owned)
    double *d_theta = nullptr;
    int32_t *d_N = nullptr;
    int32_t *d_vert_off = nullptr;
    double *d_verts = nullptr;
    double *d_radii = nullptr;           // [n_tiles * d] half-widths of the tile's box
    int32_t *d_is_box = nullptr;         // [n_tiles] 1 when the tile is its whole box
    int32_t *d_in_null = nullptr;        // [n_tiles] 1 when the tile lies in the null space
    int64_t *d_key_off = nullptr;        // [n_tiles] each tile's first key in d_keys
    int64_t *d_key_stride = nullptr;     // [n_tiles] distance between its 64-simulation chunks
    int64_t n_keys = 0;                  // key slots (sum over blocks of 64 * n_sims)
    void *d_blocks = nullptr;
    int64_t n_blocks = 0;
    WorkItem *d_items = nullptr;
    int64_t n_items = 0;
    GroupItem *d_gitems = nullptr;       // 4-arm designs
    SquareItem *d_sqitems = nullptr;     // 2-arm design
    int64_t n_gitems = 0;
    // 4-arm calibration with bracketed keys (CSE_HIER4): pilot items over the first H4_PILOT
    // simulations; per tile the bracket (lo, hi), the keys below lo, the candidates kept per region
    // ([0] the pilot's, [1 + s] item range s) and the candidate regions themselves; the tiles the
    // last selection regenerated ([0] = count)
    GroupItem *d_gitems_pilot = nullptr;
    int64_t n_gitems_pilot = 0;
    int32_t h4_maxs = 0, h4_caps = 0;    // item ranges per group (at most), candidate slots per range
    int32_t h4_max_rows = 0;             // most key rows of a block
    int64_t h4_tot = 0;                  // candidate slots per tile: H4_PCAP + h4_maxs * h4_caps
    size_t h4_cnt_alloc = 0, h4_cand_alloc = 0;   // entries of d_h4cnt / d_h4cand now allocated
    float2 *d_h4brk = nullptr;
    uint32_t *d_h4below = nullptr;
    uint32_t *d_h4cnt = nullptr;
    float *d_h4cand = nullptr;
    uint32_t *d_h4fb = nullptr;
    float h4_margin = 6.0f;              // bracket margin in standard deviations of the pilot rank
    bool h4_bracket = false;             // calibrate with bracketed keys (else every key in HBM, the f32 selection)

    // design tables (device)
    float4 *d_h4tbl = nullptr;           // 4-arm: (1 - P_1, 1 - P_2, 1 - P_3, 0) per outcome
    uint8_t *d_h4mask = nullptr;         // 4-arm designs: rejection mask at the cut per outcome
    HierNode *d_hnodes = nullptr;        // per-node constants of the hierarchical posterior
    // Phase II/III design: per-tile thresholds / configurations, the work queue
    uint32_t *d_tileT = nullptr;
    int32_t *d_cfg = nullptr;
    uint32_t *d_queue = nullptr;
    double *d_gh = nullptr;              // Gauss-Hermite nodes and weights
    unsigned long long *d_p23stats = nullptr;   // [4] work counters of the last launch
    uint8_t *d_p23look1 = nullptr;       // first-look decisions (51^4)
    WorkItem *d_p23items = nullptr;
    P23Args p23{};
    int64_t p23_grid = 0;
    int32_t p23_chunk = 256;             // simulations per queue item
    // launch shapes (cse_autotune): waves of the one-wave-per-block kernels, workgroups of the
    // group kernels
    int64_t tune_waves = 16384, tune_wgs = 16384;
    std::vector<int64_t> blk_sims;       // simulations of each block
    std::vector<int64_t> blk_row, blk_col;   // 2-arm: each block's row / column group of 8 thresholds
    std::vector<int64_t> p23_item_off;   // [n_tiles + 1] first queue item of each tile
    int64_t h4_outcomes = 0;
    double table_ms = 0.0;               // time to build the design table at platten creation
    int32_t *d_cut_tbl = nullptr;        // 2-arm: c(y0) = min{y1 : z(y0, y1) > cut}, [n+1]
    double *d_S_tbl = nullptr;           // 2-arm: S = -z per outcome y0*(n+1)+y1
    int32_t *d_S_order = nullptr;        // 2-arm: outcomes sorted by S ascending
    int32_t *d_S_group = nullptr;        // 2-arm: index of first outcome with equal S in that order
    int32_t *d_S_pos = nullptr;          // 2-arm: position of each outcome in that order
    int32_t *d_gstart = nullptr;         // 2-arm: first position of each tie group of S, [n_groups + 1]
    uint8_t *d_gcut = nullptr;           // 2-arm: per tie group g and y0, #{y1 : S(y0, y1) >= S_g}, [n_groups + 1][n + 1]
    int32_t n_groups = 0;
    float b2_margin = 5.0f;              // 2-arm selection: bracket margin in standard deviations of the count
    int32_t n_outcomes = 0;
    // 2-arm calibration: per-tile bracket of S-order positions [lo, hi] expected to hold the
    // k-th smallest statistic, and the list of tiles the bracketed selection left to the exact
    // full-histogram pass ([0] = count, then tile ids)
    int2 *d_b2br = nullptr;
    uint32_t *d_b2fb = nullptr;
    // 2-arm calibration: per block, row group u and arm-0 count y0, the cut points on y1 of the
    // row's 8 tiles as bytes: x, y = clo (S < S(lo) iff y1 >= clo), z, w = chi (S <= S(hi) iff
    // y1 >= chi); [n_blocks][8][n + 1]
    uint4 *d_b2cut = nullptr;

    std::vector<uint32_t> tile_T;        // [n_tiles * d] Bernoulli thresholds (binomial designs)

    // launch-shape generation: advanced whenever the work-item arrays a captured plan refers to are
    // rebuilt (cse_autotune), and set to PLATTEN_GONE when the platten is destroyed.  Plans hold a
    // reference to this counter and refuse to replay once it differs from its value at capture.
    std::shared_ptr<std::atomic<uint64_t>> shape_gen = std::make_shared<std::atomic<uint64_t>>(0);

    // side stream (default priority) and fork/join events of the calibration step: the
    // validation bound runs beside the selection, and in a captured graph the inversion beside
    // the simulation
    hipStream_t side = nullptr;
    // device arenas holding the read-only per-tile arrays and design tables, each filled by one
    // host-to-device copy at creation (base, bytes); the arrays point into them
    std::vector<std::pair<void *, size_t>> arenas;
    hipEvent_t ev_sim = nullptr, ev_val = nullptr, ev_fork = nullptr, ev_inv = nullptr;

    // Clopper-Pearson table: one entry per (N class, R), R = 0..N (classes = distinct N)
    int32_t n_cls = 0;
    int64_t n_cp = 0;                    // sum over classes of N + 1
    int32_t *d_cls_N = nullptr;          // [n_cls]
    int64_t *d_cls_off = nullptr;        // [n_cls] first entry of each class
    int64_t *d_cp_base = nullptr;        // [n_tiles] first entry of the tile's class
    uint32_t *d_cp_mark = nullptr;       // [n_cp] R values present in this call
    double *d_cp_tbl = nullptr;          // [n_cp]
    int32_t max_cls_N = 0;
    int32_t max_nv = 1;   // most vertices of any tile (the bound kernel's per-tile LDS rows)

    // per-tile workspaces (allocated with the platten)
    uint32_t *d_Rw = nullptr;            // rejection counts
    unsigned long long *d_Tw = nullptr;  // score sums T (binomial) [n_tiles * d]
    unsigned long long *d_Zw = nullptr;  // score sums Z (z-test), fixed point 2^-32
    double *d_apw = nullptr;             // alpha'
    int32_t *d_kw = nullptr;             // k
    double *d_lamw = nullptr;            // lambda*_i
    double *d_lamg = nullptr;            // lambda* (1)
    double *d_minpart = nullptr;         // [2 * MIN_PARTS] partial minima of the reductions over tiles
                                         // (values; for pairs, their second components after them)

    // calibration keys (allocated on first calibration): n_keys entries of 2 (outcome
    // index) or 4 (float32 statistic) bytes
    void *d_keys = nullptr;
    size_t keys_bytes = 0;
};

// error reporting
void set_error(const std::string &msg);
const char *get_error();

int build_platten(const cse_design *design, int64_t n_boxes, const double *theta,
                  const double *radii, const int32_t *sims, int32_t flags, Platten *P);
void free_platten(Platten *P);
int plan_work_items(Platten *P, int64_t target_waves);
int plan_group_items(Platten *P, int64_t target_wgs);
int h4_regions(Platten *P);
int plan_queue_items(Platten *P, int32_t chunk, int64_t grid);

}  // namespace cse

#define CSE_HIP_TRY(expr)                                                                   \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) {                                                             \
            ::cse::set_error(std::string(#expr " failed: ") + hipGetErrorString(_e));       \
            return CSE_EHIP;                                                                \
        }                                                                                   \
    } while (0)
