// Float32 division a / b by residual correction, for divisors in a bounded range.
//
// From the hardware reciprocal y0 of b, one Newton step gives y = y0 + y0 (1 - b y0); the
// quotient q0 = a y is then corrected twice with the exact residual r = a - b q (one
// fused multiply-add each): q <- q + r y (Markstein, IBM J. Res. Dev. 34(1), 1990).
// These are exactly the reciprocal, multiplies and multiply-adds of the compiler's
// correctly rounded float32 division on this GPU.  What that sequence adds are two
// operand-scaling steps, which leave both operands unchanged when
//     2^-32 <= b <= 2^32 and 2^-90 <= |a| <= 2^32
// (no denormal divisor or quotient, no tiny dividend, exponent gap below 96), and a fix-up
// of special values, which returns the corrected quotient unchanged for such operands.
// So in that range the result equals the compiler's quotient bit for bit; for a = 0 it is
// a zero whose sign may differ; for 0 < |a| < 2^-90 it stays below 2^-56 in magnitude, as
// the true quotient does.  One reciprocal serves every quotient that shares b.
//
// Host and device: the host tests drive it with reciprocal estimates around 1/b.
#pragma once

#ifndef __HIP__
#include <cmath>
#define VBH_HD
#else
#define VBH_HD __host__ __device__
#endif

namespace vbh {

// One Newton step on the reciprocal estimate y0 of 1/b.
VBH_HD inline float refine_rcp(float b, float y0) {
    const float e = fmaf(-b, y0, 1.0f);
    return fmaf(e, y0, y0);
}

// a / b from the refined reciprocal y of b.
VBH_HD inline float corrected_quotient(float a, float b, float y) {
    float q = a * y;
    float r = fmaf(-b, q, a);
    q = fmaf(r, y, q);
    r = fmaf(-b, q, a);
    return fmaf(r, y, q);
}

}  // namespace vbh
