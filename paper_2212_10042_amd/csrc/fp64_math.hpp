// fp64_math.hpp -- lean float64 exp and softplus for the bound search (device and host).
//
//  exp(x):  Cody-Waite reduction x = k ln2 + r, |r| <= ln2 / 2 (ln2 split into a 53-bit head and
//           its remainder), exp(r) by its Taylor polynomial of degree 13 (truncation < 5e-18
//           relative on that range), scaled by 2^k.  For |x| <= 700.
//  log1p(t) for 0 <= t <= 1:  log(1 + t) = 2 atanh(u), u = t / (2 + t) in [0, 1/3], by the odd
//           series 2 (u + u^3/3 + u^5/5 + ...) to u^35 (truncation < 1e-17 relative).
//  softplus(x) = log(1 + e^x) = max(x, 0) + log1p(e^-|x|).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace cse {

__host__ __device__ __forceinline__ double exp_cw(double x) {
    const double ln2_hi = 0x1.62e42fefa39efp-1;    // nearest double to ln 2
    const double ln2_lo = 0x1.abc9e3b39803fp-56;   // ln 2 - ln2_hi
    const double k = rint(x * 0x1.71547652b82fep0);  // x / ln 2
    const double r = fma(-k, ln2_lo, fma(-k, ln2_hi, x));
    double p = 1.0 / 6227020800.0;   // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// log(1 + t) = 2 atanh(u) from u = t / (2 + t) in [0, 1/3].
__host__ __device__ __forceinline__ double log1p_from_u(double u) {
    const double w = u * u;
    double s = 1.0 / 35.0;
#pragma unroll
    for (int j = 33; j >= 1; j -= 2) s = fma(s, w, 1.0 / (double)j);
    return 2.0 * u * s;
}

__host__ __device__ __forceinline__ double log1p_unit(double t) { return log1p_from_u(t / (2.0 + t)); }

__host__ __device__ __forceinline__ double softplus_fast(double x) {
    return fmax(x, 0.0) + log1p_unit(exp_cw(-fabs(x)));
}

}  // namespace cse
