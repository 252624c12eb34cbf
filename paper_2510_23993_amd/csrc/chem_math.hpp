// Exponential and logarithm on the FP32 units with FP64 range reduction (the
// mixed-precision mode), a short series for e^d - 1, and the power used by
// the step-size controllers.
#pragma once
#include <hip/hip_runtime.h>

namespace chem {

// e^x = 2^n 2^f with t = x log2(e) and n = rint(t) in FP64, f = t - n in
// [-1/2, 1/2] rounded to FP32 and exponentiated by exp2f; ~1e-7 relative.
__device__ __forceinline__ double exp32(double x) {
    const double t = x * 1.4426950408889634074;
    const double n = rint(t);
    const float f = (float)(t - n);
    return ldexp((double)exp2f(f), (int)fmax(fmin(n, 2000.0), -2000.0));
}

// ln c = (log2 m + e) ln 2 with c = m 2^e, m in [1/2, 1); c > 0
__device__ __forceinline__ double log32(double c) {
    int e;
    const double m = frexp(c, &e);
    return ((double)log2f((float)m) + (double)e) * 0.69314718055994530942;
}

// e^d - 1 for |d| < 0.35 (Taylor series to d^7; truncation below 2e-8 relative)
__device__ __forceinline__ double expm1_small(double d) {
    return d * (1.0 + d * (1.0 / 2 + d * (1.0 / 6 + d * (1.0 / 24 + d * (1.0 / 120 + d * (1.0 / 720 + d * (1.0 / 5040)))))));
}

// x^y for the BDF step-size and order controllers, which need a few digits:
// FP32 log2f and exp2f instead of the FP64 library pow (a long,
// register-hungry sequence).  x that under- or overflows FP32 gives 0 or
// inf, and the callers clamp the factors built from it to [0.2, 10], as
// they clamp the exact power.
__device__ __forceinline__ double ctl_pow(double x, double y) {
    return (double)exp2f(log2f((float)x) * (float)y);
}

}  // namespace chem
