// monopole.h -- device helpers of the monopole subtraction for plain
// backprojection (against the origin artifacts of Section 2): the slice's
// mass from the partial sinogram sums, and e^-x I0(x) for the closed-form
// backprojection of the subtracted Gaussian.
#pragma once

#include "bst_internal.h"

namespace bst {

// m = mono_inv * sum of the slice's kMassChunks partial sums, added in one
// fixed order, so the spectrum and row kernels obtain the same value.
__device__ inline float monopole_mass(const float* part, int s, float mono_inv) {
    const float* ps = part + (size_t)s * kMassChunks;
    float acc = 0.f;
#pragma unroll 8
    for (int c = 0; c < kMassChunks; ++c) acc += ps[c];
    return acc * mono_inv;
}

// e^-x I0(x) for x >= 0 from the polynomial approximations of Abramowitz and
// Stegun, Handbook of Mathematical Functions, 9.8.1 (x <= 3.75, absolute error
// of I0 below 1.6e-7) and 9.8.2 (x > 3.75, absolute error of
// sqrt(x) e^-x I0(x) below 1.9e-7).
__device__ inline float scaled_bessel_i0(float x) {
    if (x <= 3.75f) {
        const float t = x * (1.0f / 3.75f);
        const float y = t * t;
        const float i0 = 1.0f + y * (3.5156229f + y * (3.0899424f + y * (1.2067492f + y * (0.2659732f +
                                     y * (0.0360768f + y * 0.0045813f)))));
        return i0 * expf(-x);
    }
    const float y = 3.75f / x;
    const float p = 0.39894228f + y * (0.01328592f + y * (0.00225319f + y * (-0.00157565f + y * (0.00916281f +
                    y * (-0.02057706f + y * (0.02635537f + y * (-0.01647633f + y * 0.00392377f)))))));
    return p * rsqrtf(x);
}

}  // namespace bst
