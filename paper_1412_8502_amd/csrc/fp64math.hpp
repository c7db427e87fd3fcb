// FP64 exp on the non-positive half-line and FP64 reciprocal square root for
// the pair kernels, written from textbook methods:
//   exp: Cody-Waite range reduction x = k ln2 + r, |r| <= ln2/2, with ln2
//        split into a 32-bit head (so k * head is exact for |k| < 2^21) and
//        a tail, then the degree-13 Taylor polynomial of e^r by Horner's
//        rule (truncation below 4e-18 on |r| <= 0.347) and a scaling by 2^k.
//        Only x in [-700, 0] occurs here (e^{-r^2/2Lambda} inside the
//        nuclear cutoff, e^{-r/lambda} inside the box); no overflow, NaN or
//        infinity handling.
//   rsqrt: the hardware estimate refined by two Newton-Raphson steps
//        y <- y + (y/2)(1 - x y^2).
// Both are __host__ __device__ so a host build can check them against libm.
#pragma once

#include <cmath>

#ifndef __HIP_DEVICE_COMPILE__
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

namespace pasta {

__host__ __device__ inline double exp_nonpos(double x)
{
    const double log2e = 1.4426950408889634;
    const double ln2_hi = 0x1.62e42ff000000p-1;   // ln 2 to 32 bits
    const double ln2_lo = -0x1.718432a1b0e26p-35;  // ln 2 - ln2_hi
    x = x < -700.0 ? -700.0 : x;
    const double k = rint(x * log2e);
    double r = fma(-k, ln2_hi, x);
    r = fma(-k, ln2_lo, r);
    double p = 1.6059043836821613e-10;   // 1/13!
    p = fma(p, r, 2.08767569878681e-09);  // 1/12!
    p = fma(p, r, 2.505210838544172e-08);
    p = fma(p, r, 2.755731922398589e-07);
    p = fma(p, r, 2.7557319223985893e-06);
    p = fma(p, r, 2.48015873015873e-05);
    p = fma(p, r, 0.0001984126984126984);
    p = fma(p, r, 0.001388888888888889);
    p = fma(p, r, 0.008333333333333333);
    p = fma(p, r, 0.041666666666666664);
    p = fma(p, r, 0.16666666666666666);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// Newton-Raphson refinement of an estimate y of 1/sqrt(x) (x > 0).
__host__ __device__ inline double rsqrt_refine(double x, double y)
{
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);  // 1 - x y^2
        y = fma(0.5 * y, e, y);
    }
    return y;
}

__host__ __device__ inline double rsqrt_fast(double x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return rsqrt_refine(x, __builtin_amdgcn_rsq(x));
#else
    return 1.0 / std::sqrt(x);
#endif
}

}  // namespace pasta
