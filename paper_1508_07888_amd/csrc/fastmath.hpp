// fastmath.hpp -- double-precision exp and log for the chemistry rates.
//
// The rate fits need about a dozen exp/log evaluations per substep.  The
// general-purpose library versions carry extra-precision steps (double-double
// log, full special-case handling) that this use does not need; these keep
// ~1 ulp accuracy over the arguments the rates produce (finite, log of a
// positive normal number) in roughly a third of the instructions.
//
//  exp:  Cody-Waite reduction x = k ln2 + r (ln2 split in a high part with
//        trailing zero bits and a low part), |r| <= ln2/2, Taylor series of
//        e^r to degree 13 (truncation < 5e-18), scaled by 2^k.  Arguments are
//        clamped to [-745.2, 709.78] (the result is 0 below; the rates never
//        exceed the upper end).
//  log:  x = m 2^e with m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1),
//        ln m = 2 atanh s = 2 (s + s^3/3 + ... + s^23/23) (|s| < 0.172,
//        truncation < 1e-19), plus e ln2 in the same split form.
#pragma once

#include <hip/hip_runtime.h>

namespace emma {

__host__ __device__ __forceinline__ double exp_fp64(double x) {
    const double log2e = 1.4426950408889634074;
    const double ln2_hi = 6.93147180369123816490e-01;  // 0x3FE62E42FEE00000
    const double ln2_lo = 1.90821492927058770002e-10;
    // branch-free range clamp: above it the value would overflow (never reached
    // by the rates), below it 2^k underflows to exactly zero
    x = fmin(fmax(x, -745.2), 709.78);
    const double k = rint(x * log2e);
    double r = fma(-k, ln2_hi, x);
    r = fma(-k, ln2_lo, r);
    // Horner form of sum_{n<=13} r^n / n!
    double p = 1.0 / 6227020800.0;          // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);       // 1/12!
    p = fma(p, r, 1.0 / 39916800.0);        // 1/11!
    p = fma(p, r, 1.0 / 3628800.0);         // 1/10!
    p = fma(p, r, 1.0 / 362880.0);          // 1/9!
    p = fma(p, r, 1.0 / 40320.0);           // 1/8!
    p = fma(p, r, 1.0 / 5040.0);            // 1/7!
    p = fma(p, r, 1.0 / 720.0);             // 1/6!
    p = fma(p, r, 1.0 / 120.0);             // 1/5!
    p = fma(p, r, 1.0 / 24.0);              // 1/4!
    p = fma(p, r, 1.0 / 6.0);               // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// 1/d: hardware reciprocal estimate refined by two Newton steps on the device
// (relative error ~1 ulp; used where an exactly rounded quotient is not needed).
__host__ __device__ __forceinline__ double recip_fp64(double d) {
#ifdef __HIP_DEVICE_COMPILE__
    double q = __builtin_amdgcn_rcp(d);
    double t = fma(-d, q, 1.0);
    q = fma(q, t, q);
    t = fma(-d, q, 1.0);
    return fma(q, t, q);
#else
    return 1.0 / d;
#endif
}

__host__ __device__ __forceinline__ double log_fp64(double x) {
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) * recip_fp64(m + 1.0);
    const double s2 = s * s;
    // 2 atanh(s) = 2 s sum_{j<=11} s^(2j) / (2j+1)
    double p = 1.0 / 23.0;
    p = fma(p, s2, 1.0 / 21.0);
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double lm = 2.0 * s + 2.0 * s * s2 * p;
    const double de = (double)e;
    return fma(de, ln2_hi, fma(de, ln2_lo, lm));
}

}  // namespace emma
