// fastmath.hpp -- double-precision exp and log for the chemistry rates.
//
// The rate fits need about a dozen exp/log evaluations per substep.  The
// general-purpose library versions carry extra-precision steps (double-double
// log, full special-case handling) that this use does not need; these keep
// ~1 ulp accuracy over the arguments the rates produce (finite, log of a
// positive normal number) in roughly a third of the instructions.
//
//  exp:  Cody-Waite reduction x = k ln2 + r (ln2 split in a high part with
//        trailing zero bits and a low part), |r| <= ln2/2, a degree-11
//        polynomial for e^r (the Chebyshev interpolant on that interval,
//        error 3.2e-18), scaled by 2^k.  Arguments are clamped to
//        [-745.2, 709.78] (the result is 0 below; the rates never exceed the
//        upper end).
//  log:  x = m 2^e with m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1),
//        ln m = 2 atanh s = 2 s + 2 s^3 p(s^2) (|s| < 0.172) with p a degree-6
//        polynomial (Chebyshev interpolant of (atanh s / s - 1) / s^2, error
//        1.6e-16 in p, below 5e-18 relative to ln m), plus e ln2 in the same
//        split form.
// The coefficients are printed by fastmath_coeffs.py (50-digit arithmetic).
// Measured against 64-bit-mantissa references on 2e7 arguments: exp within
// 0.94 ulp, log within 0.93 ulp where |ln x| >= 1 and 1.5e-16 absolute below.
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
    double p = 0x1.af635e4f6b5eep-26;
    p = fma(p, r, 0x1.28b43a93fe57ap-22);
    p = fma(p, r, 0x1.71ddf5514be0cp-19);
    p = fma(p, r, 0x1.a01991731e6fap-16);
    p = fma(p, r, 0x1.a01a01b150ad2p-13);
    p = fma(p, r, 0x1.6c16c1881156bp-10);
    p = fma(p, r, 0x1.111111110f205p-7);
    p = fma(p, r, 0x1.555555554f067p-5);
    p = fma(p, r, 0x1.555555555555ap-3);
    p = fma(p, r, 0x1.0000000000011p-1);
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
    double p = 0x1.2b61a9651d276p-4;
    p = fma(p, s2, 0x1.39fd9e34422d0p-4);
    p = fma(p, s2, 0x1.7462ba83c0355p-4);
    p = fma(p, s2, 0x1.c71c62d0f22d4p-4);
    p = fma(p, s2, 0x1.2492492e01697p-3);
    p = fma(p, s2, 0x1.9999999995250p-3);
    p = fma(p, s2, 0x1.5555555555558p-2);
    const double lm = 2.0 * s + 2.0 * s * s2 * p;
    const double de = (double)e;
    return fma(de, ln2_hi, fma(de, ln2_lo, lm));
}

}  // namespace emma
