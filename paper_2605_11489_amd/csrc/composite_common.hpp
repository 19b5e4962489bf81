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
//   s0 = (mu, mv, a, b), s1 = (c, lo, A, B), s2 = (C, r, g, b), s3 = (z, -, -, -)
// mu, mv: 2D mean relative to the tile origin, formed in FP64 and rounded
// once, so the float offset to a pixel centre keeps full precision;
// A, B, C: conic; a, b, c = -log2(e)/2 times A, B, C and lo = log2(opacity),
// so the exponent of alpha' in base 2 is
//   e = dx (a dx + b dy) + dy (b dx + c dy) + lo,
// whose two slopes a dx + b dy and b dx + c dy are -log2(e)/2 times the
// terms A dx + B dy and B dx + C dy of alpha's pixel gradient (Eq. 3).
struct Staged {
    float4 s0, s1, s2, s3;
};

__device__ __forceinline__ Staged stage_gaussian(const GaussRec& r, double x0, double y0) {
    Staged s;
    s.s0 = make_float4((float)(r.u - x0), (float)(r.v - y0), -0.5f * kLog2e * r.A, -0.5f * kLog2e * r.B);
    s.s1 = make_float4(-0.5f * kLog2e * r.C, __log2f(r.o), r.A, r.B);
    s.s2 = make_float4(r.C, r.r, r.g, r.b);
    s.s3 = make_float4(r.z, 0.f, 0.f, 0.f);
    return s;
}

// Base-2 exponent of alpha' at the pixel offset (dx, dy) = mean - pixel, and
// its two slopes (s0, s1 as staged; c1 = (c, lo)).
__device__ __forceinline__ float alpha_exponent_slopes(const float4& s0, const float2& c1, float dx, float dy,
                                                       float& ga, float& gb) {
    ga = __builtin_fmaf(s0.z, dx, s0.w * dy);
    gb = __builtin_fmaf(s0.w, dx, c1.x * dy);
    return __builtin_fmaf(dx, ga, __builtin_fmaf(dy, gb, c1.y));
}

__device__ __forceinline__ float alpha_exponent(const float4& s0, const float4& s1, float dx, float dy) {
    float ga, gb;
    return alpha_exponent_slopes(s0, make_float2(s1.x, s1.y), dx, dy, ga, gb);
}

// A dx + B dy = kSlopeToConic times the slope a dx + b dy (-2 ln 2)
constexpr float kSlopeToConic = -1.3862943611198906f;

__device__ __forceinline__ float fast_exp2(float e) { return __builtin_amdgcn_exp2f(e); }

// Which 8x8 quadrants of the tile (bit w for quadrant x >= 8 ? 1 : 0 plus
// y >= 8 ? 2 : 0) can hold a pixel centre where the Gaussian reaches
// alpha' >= 1/255.  That region is the ellipse q(d) <= Q with
// Q = 2 ln(255 o); its bounding box has half-widths sqrt(Q Sigma'_xx) and
// sqrt(Q Sigma'_yy), Sigma' being the inverse of the conic.  The test is
// conservative: Q carries a 0.1 % + 1e-3 margin and the half-widths 0.1 % +
// 0.02 px, far above both the float32 error of the box itself and that of the
// per-pixel exponent.  The latter is bounded because conics with
// B^2 > 0.996 AC are never culled: otherwise |A dx^2| + |2B dx dy| + |C dy^2|
// stays within 1000 q, so near the threshold (q <= 11.1) the exponent's
// rounding error is about 2e-3 against a margin of about 0.017.  A cleared
// bit therefore only removes (Gaussian, pixel) pairs that the per-pixel test
// would skip anyway.
// A quadrant whose box passes is then tested exactly: the minimum of q over
// the rectangle spanned by its pixel centres (zero when the mean lies inside,
// else the smallest of the four edge minima, each a clamped 1-D quadratic)
// must not exceed the same Q.  The float32 error of q near Q is bounded by
// the same conditioning limit, far below the margins.  For thin, rotated
// ellipses this drops a fifth of the quadrants the box keeps.
__device__ __forceinline__ float edge_min_q(float A, float B, float C, float X, float Y0, float Y1, float nBoC) {
    // min over y in [Y0, Y1] of A X^2 + 2 B X y + C y^2: at y = -B X / C, clamped
    const float y = fminf(fmaxf(nBoC * X, Y0), Y1);
    return __builtin_fmaf(A * X, X, y * __builtin_fmaf(2.f * B, X, C * y));
}

__device__ __forceinline__ uint32_t quadrant_mask(const GaussRec& r, float mu, float mv, float lo) {
    if (lo < kLog2AlphaMin - 1e-3f) return 0u;
    const float Q = fmaxf(2.f * (lo - kLog2AlphaMin) * (1.f / kLog2e), 0.f) * 1.001f + 1e-3f;
    const float A = r.A, B = r.B, C = r.C;
    const float ac = A * C, det = ac - B * B;
    if (!(A > 0.f) || !(C > 0.f) || !(det > 4e-3f * ac)) return 0xFu;
    const float qd = Q / det;
    const float xe = __builtin_sqrtf(qd * C) * 1.001f + 0.02f;
    const float ye = __builtin_sqrtf(qd * A) * 1.001f + 0.02f;
    const float nBoC = -B / C, nBoA = -B / A;
    uint32_t m = 0;
#pragma unroll 1
    for (int w = 0; w < 4; ++w) {   // (not unrolled: the compositing kernels' register budget)
        const float qx0 = (float)((w & 1) * 8) + 0.5f, qy0 = (float)((w >> 1) * 8) + 0.5f;
        if (!(mu + xe >= qx0 && mu - xe <= qx0 + 7.f && mv + ye >= qy0 && mv - ye <= qy0 + 7.f)) continue;
        // the pixel centres' rectangle relative to the mean
        const float X0 = qx0 - mu, X1 = qx0 + 7.f - mu, Y0 = qy0 - mv, Y1 = qy0 + 7.f - mv;
        const bool inside = X0 <= 0.f && X1 >= 0.f && Y0 <= 0.f && Y1 >= 0.f;
        const float qx = fminf(edge_min_q(A, B, C, X0, Y0, Y1, nBoC), edge_min_q(A, B, C, X1, Y0, Y1, nBoC));
        const float qy = fminf(edge_min_q(C, B, A, Y0, X0, X1, nBoA), edge_min_q(C, B, A, Y1, X0, X1, nBoA));
        if (inside || fminf(qx, qy) <= Q) m |= 1u << w;
    }
    return m;
}

}  // namespace gs
