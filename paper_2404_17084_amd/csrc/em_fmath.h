// FP32 elementary functions of the mixed-precision edge terms (device only).
//
// The FP32 terms are accumulated in FP64 and checked against an FP64 oracle at
// 1e-5 relative per cell, so a few ulp per function are enough; these forms
// replace the correctly rounded library versions, which cost 3-6 times the
// instructions.  Domains are restricted to what the edge terms use.
#pragma once

#include <hip/hip_runtime.h>

namespace em {

// Hardware square root and reciprocal (about 1 ulp).  Arguments of the edge
// terms are 0 or above 2^-100, so no denormal rescaling is needed.
__device__ __forceinline__ float sqrt_f32(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rcp_f32(float x) { return __builtin_amdgcn_rcpf(x); }

// atan2(y, x) for y >= 0, result in [0, pi]; (0, 0) gives 0.
// With t = min(|x|, y) / max(|x|, y) in [0, 1], atan t = t P(t^2), P of degree
// 8 fitted for least maximum relative error on [0, 1] (Lawson's iteratively
// reweighted least squares; fit error 1.6e-8), then pi/2 - r when y > |x| and
// pi - r when x < 0.  Within 4 ulp of atan2 with a 1-ulp reciprocal.
__device__ __forceinline__ float atan2_f32(float y, float x)
{
    const float ax = fabsf(x);
    const bool steep = y > ax;  // selects instead of fminf/fmaxf (no NaN handling needed here)
    const float mn = steep ? ax : y, mx = steep ? y : ax;
    const float t = mx > 0.0f ? mn * rcp_f32(mx) : 0.0f;
    const float z = t * t;
    float p = 0.0028501402121037245f;
    p = fmaf(p, z, -0.016069695353507996f);
    p = fmaf(p, z, 0.04269338771700859f);
    p = fmaf(p, z, -0.07504468411207199f);
    p = fmaf(p, z, 0.10641025751829147f);
    p = fmaf(p, z, -0.14203672111034393f);
    p = fmaf(p, z, 0.1999262422323227f);
    p = fmaf(p, z, -0.33333075046539307f);
    p = fmaf(p, z, 1.0f);
    float r = t * p;
    r = steep ? 1.5707963267948966f - r : r;
    return x < 0.0f ? 3.141592653589793f - r : r;
}

// log(1 + u) for u >= 0 (u = 0 gives 0).  1 + u = 2^k m with m in
// [sqrt(1/2), sqrt(2)), f = m - 1 (exact), log m = 2 atanh(s) with
// s = f / (2 + f), |s| <= 0.172, by its series through s^9 (truncation below
// 1e-9 relative).  When 1 + u < 2 the rounding error of 1 + u, u - ((1 + u) - 1),
// is exact and is added back to first order.  Within 5 ulp of log1p with a
// 1-ulp reciprocal.
__device__ __forceinline__ float log1p_f32(float u)
{
    const float v = 1.0f + u;
    int k = __builtin_amdgcn_frexp_expf(v);
    float m = __builtin_amdgcn_frexp_mantf(v);
    if (m < 0.70710678f) {
        m += m;
        k -= 1;
    }
    const float f = m - 1.0f;
    const float s = f * rcp_f32(2.0f + f);
    const float s2 = s * s;
    float p = fmaf(s2, 1.0f / 9.0f, 1.0f / 7.0f);
    p = fmaf(p, s2, 1.0f / 5.0f);
    p = fmaf(p, s2, 1.0f / 3.0f);
    p = fmaf(p, s2, 1.0f);
    const float corr = v < 2.0f ? (u - (v - 1.0f)) * rcp_f32(v) : 0.0f;
    return fmaf((float)k, 0.6931471805599453f, fmaf(s + s, p, corr));
}

}  // namespace em
