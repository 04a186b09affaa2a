// gelu.hpp -- GELU and its derivative for the closure network, with the normal
// CDF through erf by Abramowitz and Stegun, Handbook of Mathematical
// Functions, formula 7.1.26: for y >= 0
//     erf y = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) exp(-y^2),
//     t = 1 / (1 + p y),
// with an absolute error of at most 1.5e-7 (erf is odd for y < 0).  Evaluated
// in binary32 the cancellation in 1 - (...) exp(-y^2) near y = 0 raises the
// error to about 6e-7 absolute, which moves GELU by less than 1e-6 of its
// value: three orders of magnitude below the BF16 rounding of the
// activations that follows.  On the GPU the reciprocal and the exponential are
// the hardware's approximations; compiled for the host (the tests), plain
// division and exp2f.  Plain C++ otherwise, like fmath.hpp.
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

// erf y; *ex receives exp(-y^2), which the derivative of GELU reuses.
LBMPCD_HD float erf_as(float y, float* ex) {
    const float a = fabsf(y);
    const float d = fmaf(0.3275911f, a, 1.0f);
#if defined(__HIP_DEVICE_COMPILE__)
    const float t = __builtin_amdgcn_rcpf(d);
    const float e = __builtin_amdgcn_exp2f(-(a * a) * 1.44269504088896341f);  // exp(-a^2)
#else
    const float t = 1.0f / d;
    const float e = exp2f(-(a * a) * 1.44269504088896341f);
#endif
    float p = 1.061405429f;
    p = fmaf(p, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    p *= t;
    *ex = e;
    return copysignf(fmaf(-p, e, 1.0f), y);
}

// GELU x Phi(x), Phi the normal CDF (1 + erf(x / sqrt 2)) / 2.
LBMPCD_HD float gelu(float x) {
    float e;
    return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f, &e));
}

// Its derivative Phi(x) + x phi(x), phi(x) = exp(-x^2 / 2) / sqrt(2 pi).
LBMPCD_HD float gelu_grad(float x) {
    float e;
    const float cdf = 0.5f * (1.0f + erf_as(x * 0.70710678118654752f, &e));
    return cdf + x * (0.39894228040143268f * e);
}

}  // namespace lbmpcd
