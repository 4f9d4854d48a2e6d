// 64-bit fixed-point sums for the LDS gradient scatters.  Integer LDS adds
// (ds_add_u64) run ~1.9x faster than FP64 ones on gfx950, and integer sums
// are exact and independent of the order of the adds.  A scatter takes a
// power-of-two scale from a bound on its terms, such that every term stays
// below 2^50 and every sum of at most n terms below 2^61.
#pragma once

#include "pdfx_internal.h"

namespace pdfx {

// Larger of a and b; NaN if either is NaN.
__device__ __forceinline__ double nan_max(double a, double b)
{
    return (b > a || b != b) ? b : a;
}

// Bound on the sum of |folded weights| over t in [0, 1] for one interval.
__device__ __forceinline__ double weight_sum_bound(const IntervalRec<double> &r)
{
    return 1.0 + (4.0 / 27.0) * (fabs(r.pl) + fabs(r.plql) + fabs(r.ql) + fabs(r.qr) +
                                 fabs(r.qrpr) + fabs(r.pr));
}

// Round-to-nearest fixed point of c * f (|c * f| < 2^51): adding 1.5 * 2^52
// leaves the integer in the low mantissa bits.
__device__ __forceinline__ unsigned long long to_fixed(double c, double f)
{
    const double t = fma(c, f, 6755399441055744.0);
    return (unsigned long long)(__double_as_longlong(t) - 0x4338000000000000LL);
}

// Fixed-point exponent for terms bounded by bnd, summed at most n at a time.
// Kept within [-1000, 1000], so that 2^S and 2^-S are normal doubles; bounds
// below ~2^-950 then give terms that round to 0.
__device__ __forceinline__ int fixed_exponent(double bnd, int64_t n)
{
    int lc, lb;
    frexp((double)n, &lc);   // n < 2^lc
    frexp(bnd, &lb);         // bnd < 2^lb (0 for bnd = 0)
    const int smax = 61 - lc < 50 ? 61 - lc : 50;
    const int e = smax - lb;
    return e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
}

}  // namespace pdfx
