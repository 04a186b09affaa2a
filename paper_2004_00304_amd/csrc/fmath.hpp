// fmath.hpp -- the two elementary functions of the Box-Muller transform in
// FP64, on the domains the transform actually uses, without library calls.
// Plain C++ (no HIP types), so that the same source is also compiled for the
// host and checked against the C library there.
//
//   ln x, x in (0, 1]:  x = m 2^e with m in [sqrt(1/2), sqrt(2)); then
//     ln m = 2 atanh s with s = (m - 1) / (m + 1), |s| < 0.1716, summed as
//     2 s (1 + s^2/3 + s^4/5 + ... + s^20/21); the first omitted term is below
//     2^-56 of the sum.
//   sin and cos of 2 pi u, u in [0, 1):  4u = q + f exactly, with q = rint(4u)
//     and |f| <= 1/2, so the angle is q pi/2 + y with y = f pi/2, |y| <= pi/4;
//     sin y and cos y by their Taylor series to the y^15 and y^16 terms (the
//     first omitted terms are below 5e-17 and 3e-18 on that interval), then
//     the quadrant q mod 4 swaps and negates them.
// Both are accurate to a few units in the last place, which is what the FP64
// path needs (the C library's versions differ from each other by as much).
//
// The binary32 pair (for particles stored in binary32) follows a fixed
// definition, every step one IEEE binary32 operation, so that it is bit-exact
// wherever it is evaluated:
//   ln x, x in (0, 1]:  m in [sqrt(1/2), sqrt(2)) as above; 2 atanh s summed as
//     2 s (1 + z/3 + z^2/5 + z^3/7 + z^4/9), z = s^2 (first omitted term below
//     2e-9 of the sum); ln 2 and sqrt(1/2) rounded to binary32.
//   sin and cos of 2 pi u:  the same quadrant reduction with pi/2 rounded to
//     binary32; sin y to y^9/9!, cos y to y^8/8! (first omitted terms below
//     2e-9 and 2.5e-8 for |y| <= pi/4).
#pragma once

#include <math.h>

#ifndef LBMPCD_HD
#if defined(__HIPCC__)
#define LBMPCD_HD __host__ __device__ __forceinline__
#else
#define LBMPCD_HD inline
#endif
#endif

namespace lbmpcd {

LBMPCD_HD double ln_unit(double x) {
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752) {
        m = m + m;
        e -= 1;
    }
    const double f = m - 1.0;  // exact: m is within a factor two of one
    const double s = f / (2.0 + f);
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double two_s = s + s;
    const double lm = fma(two_s * z, p, two_s);  // 2 s (1 + z p)
    return fma((double)e, 0.69314718055994531, lm);
}

LBMPCD_HD void sincos_2pi(double u, double* sn, double* cs) {
    const double t = 4.0 * u;
    const double q = rint(t);
    const double y = (t - q) * 1.5707963267948966;  // t - q is exact
    const double z = y * y;
    double ps = -1.0 / 1307674368000.0;  // -1/15!
    ps = fma(ps, z, 1.0 / 6227020800.0);  // 1/13!
    ps = fma(ps, z, -1.0 / 39916800.0);   // -1/11!
    ps = fma(ps, z, 1.0 / 362880.0);      // 1/9!
    ps = fma(ps, z, -1.0 / 5040.0);       // -1/7!
    ps = fma(ps, z, 1.0 / 120.0);         // 1/5!
    ps = fma(ps, z, -1.0 / 6.0);          // -1/3!
    const double S = fma(ps * z, y, y);
    double pc = 1.0 / 20922789888000.0;   // 1/16!
    pc = fma(pc, z, -1.0 / 87178291200.0);  // -1/14!
    pc = fma(pc, z, 1.0 / 479001600.0);     // 1/12!
    pc = fma(pc, z, -1.0 / 3628800.0);      // -1/10!
    pc = fma(pc, z, 1.0 / 40320.0);         // 1/8!
    pc = fma(pc, z, -1.0 / 720.0);          // -1/6!
    pc = fma(pc, z, 1.0 / 24.0);            // 1/4!
    pc = fma(pc, z, -0.5);                  // -1/2!
    const double C = fma(pc, z, 1.0);
    const int qm = (int)q & 3;
    const double a = (qm & 1) ? C : S;  // sin of the angle up to sign
    const double b = (qm & 1) ? S : C;  // cos of the angle up to sign
    *sn = (qm & 2) ? -a : a;
    *cs = (qm == 1 || qm == 2) ? -b : b;
}

LBMPCD_HD float ln_unit32(float x) {
    int e;
    float m = frexpf(x, &e);  // x = m 2^e, m in [1/2, 1)
    if (m < 0x1.6a09e6p-1f) {  // sqrt(1/2) in binary32
        m = m + m;
        e -= 1;
    }
    const float f = m - 1.0f;  // exact
    const float s = f / (2.0f + f);
    const float z = s * s;
    float p = 1.0f / 9.0f;
    p = fmaf(p, z, 1.0f / 7.0f);
    p = fmaf(p, z, 1.0f / 5.0f);
    p = fmaf(p, z, 1.0f / 3.0f);
    const float two_s = s + s;
    const float lm = fmaf(two_s * z, p, two_s);
    return fmaf((float)e, 0x1.62e430p-1f, lm);  // ln 2 in binary32
}

LBMPCD_HD void sincos_2pi32(float u, float* sn, float* cs) {
    const float t = 4.0f * u;
    const float q = rintf(t);
    const float y = (t - q) * 0x1.921fb6p+0f;  // pi/2 in binary32; t - q is exact
    const float z = y * y;
    float ps = 1.0f / 362880.0f;       // 1/9!
    ps = fmaf(ps, z, -1.0f / 5040.0f);  // -1/7!
    ps = fmaf(ps, z, 1.0f / 120.0f);    // 1/5!
    ps = fmaf(ps, z, -1.0f / 6.0f);     // -1/3!
    const float S = fmaf(ps * z, y, y);
    float pc = 1.0f / 40320.0f;         // 1/8!
    pc = fmaf(pc, z, -1.0f / 720.0f);   // -1/6!
    pc = fmaf(pc, z, 1.0f / 24.0f);     // 1/4!
    pc = fmaf(pc, z, -0.5f);            // -1/2!
    const float C = fmaf(pc, z, 1.0f);
    const int qm = (int)q & 3;
    const float a = (qm & 1) ? C : S;
    const float b = (qm & 1) ? S : C;
    *sn = (qm & 2) ? -a : a;
    *cs = (qm == 1 || qm == 2) ? -b : b;
}

}  // namespace lbmpcd
