// kernels.h -- launchers of the device kernels (library-internal).
#pragma once
#include "cse_internal.h"

namespace cse {

hipError_t launch_binom2(const Platten &P, uint64_t seed, uint32_t *R, unsigned long long *sumT,
                         uint4 *recs, hipStream_t st);
hipError_t launch_ztest1(const Platten &P, uint64_t seed, uint32_t *R, unsigned long long *sumZfx,
                         float *keys, hipStream_t st);
hipError_t launch_plain_tile(const Platten &P, uint64_t seed, int64_t t, uint32_t T0, uint32_t T1,
                             uint32_t *R_tile, hipStream_t st);
hipError_t launch_bound(const Platten &P, int mode, const uint32_t *R, const double *a_in,
                        double level, double *out, double *q_out, int32_t *k_out, double *cp_out,
                        hipStream_t st);
hipError_t launch_select(const Platten &P, const void *keys, const int32_t *k, double *lam, int32_t *rej_at,
                         hipStream_t st);
hipError_t launch_b2_bracket(const Platten &P, const int32_t *k, hipStream_t st);
hipError_t launch_min(const Platten &P, const double *v, const int32_t *in_null, int64_t n, double *out,
                      hipStream_t st);
hipError_t launch_tiebreak(const Platten &P, uint64_t seed, const int32_t *k, const double *lam, int32_t *rej_at,
                           uint32_t *c_tile, hipStream_t st);
hipError_t launch_min_pair(const Platten &P, const double *v, const uint32_t *c, const int32_t *in_null, int64_t n,
                           double *out_v, uint32_t *out_c, hipStream_t st);
hipError_t launch_confset(const Platten &P, const double *s_obs, int64_t s_stride, const double *lam,
                          const double *coef, int link, int32_t *keep, double *e_lo, double *e_hi,
                          double *e_range, hipStream_t st);
hipError_t launch_finish(const Platten &P, const uint32_t *R, const unsigned long long *sumT,
                         const unsigned long long *sumZfx, int32_t *R_out, int64_t *T_out,
                         double *Z_out, double *grad, hipStream_t st);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
hipError_t launch_taylor(const Platten &P, const double *f, const double *g, double *bound, int32_t *vertex,
                         double *point, hipStream_t st);
hipError_t launch_hier4_table(int n, float4 *tbl, const HierNode *nodes, hipStream_t st);
hipError_t launch_h4_mask(const float4 *tbl, int64_t n, float cut, int nbits, uint8_t *mask, hipStream_t st);
hipError_t launch_basket_table(int n, const double *theta0, float4 *tbl, const HierNode *nodes, hipStream_t st);
// pass: H4_PASS_ALL every simulation (keys: float32 keys of all of them, or none); H4_PASS_PILOT the
// first H4_PILOT simulations with float32 keys; H4_PASS_MAIN the rest, bracketed keys (4-arm design)
enum { H4_PASS_ALL = 0, H4_PASS_PILOT = 1, H4_PASS_MAIN = 2 };
hipError_t launch_hier4(const Platten &P, uint64_t seed, uint32_t *R, unsigned long long *sumT, float *keys,
                        hipStream_t st, int pass = H4_PASS_ALL);
// bracketed 4-arm selection: brackets from the pilot keys (after k is known), then, after the
// main pass, lambda*_i and the count below it (exact; tiles whose k-th key is not among the
// candidates regenerate their keys from the counter-based generator)
hipError_t launch_h4_bracket(const Platten &P, const float *keys, const int32_t *k, double *lam, int32_t *rej_at,
                             hipStream_t st);
hipError_t launch_h4_select(const Platten &P, uint64_t seed, const int32_t *k, double *lam, int32_t *rej_at,
                            hipStream_t st);
hipError_t launch_phase23(const Platten &P, uint64_t seed, uint32_t *R, unsigned long long *sumT, float *keys,
                          hipStream_t st);
hipError_t launch_p23_look1(const Platten &P, hipStream_t st);
hipError_t launch_phase23_items(const Platten &P, uint64_t seed, const WorkItem *items, int64_t n_items, int64_t grid,
                                uint32_t *R, hipStream_t st);
hipError_t launch_phase23_tile(const Platten &P, uint64_t seed, int64_t t, uint32_t *R_tile, hipStream_t st);
hipError_t launch_hier4_plain(const Platten &P, uint64_t seed, int64_t t, uint32_t *R_tile, hipStream_t st);

}  // namespace cse
