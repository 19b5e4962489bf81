// Per-(Gaussian, tile) staging and per-pixel alpha evaluation shared by the
// forward and backward compositing kernels, so both take every skip / stop /
// clamp decision on bit-identical float32 values.
#pragma once

#include "gs_common.hpp"

namespace gs {

constexpr float kLog2e = 1.4426950408889634f;
// alpha' = exp2(e) >= 1/255  <=>  e >= log2(1/255)
constexpr float kLog2AlphaMin = -7.994353436858858f;

// A Gaussian as one 16x16 tile sees it, four float4 in LDS:
//   s0 = (mu, mv, a2, b2), s1 = (c2, lo, A, B), s2 = (C, r, g, b), s3 = (z, -, -, -)
// mu, mv: 2D mean relative to the tile origin, formed in FP64 and rounded
// once, so the float offset to a pixel centre keeps full precision;
// A, B, C: conic; a2 = -A log2(e)/2, b2 = -B log2(e), c2 = -C log2(e)/2 and
// lo = log2(opacity), so the exponent of alpha' in base 2 is
//   e = a2 dx^2 + b2 dx dy + c2 dy^2 + lo.
struct Staged {
    float4 s0, s1, s2, s3;
};

__device__ __forceinline__ Staged stage_gaussian(const GaussRec& r, double x0, double y0) {
    Staged s;
    s.s0 = make_float4((float)(r.u - x0), (float)(r.v - y0), -0.5f * kLog2e * r.A, -kLog2e * r.B);
    s.s1 = make_float4(-0.5f * kLog2e * r.C, __log2f(r.o), r.A, r.B);
    s.s2 = make_float4(r.C, r.r, r.g, r.b);
    s.s3 = make_float4(r.z, 0.f, 0.f, 0.f);
    return s;
}

// Base-2 exponent of alpha' at the pixel offset (dx, dy) = mean - pixel.
__device__ __forceinline__ float alpha_exponent(const float4& s0, const float4& s1, float dx, float dy) {
    const float m = s0.w * dy;
    const float n = __builtin_fmaf(s0.z, dx, m);
    const float k = s1.x * dy;
    const float l = __builtin_fmaf(k, dy, s1.y);
    return __builtin_fmaf(dx, n, l);
}

__device__ __forceinline__ float fast_exp2(float e) { return __builtin_amdgcn_exp2f(e); }

}  // namespace gs
