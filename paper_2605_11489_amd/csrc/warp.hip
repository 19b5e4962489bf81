// Pose-derived motion vectors and forward warping of a rendered frame to
// another camera (3DGS^3 Sec. 4.2, Eq. 12 and Eq. 13).
//
// Eq. 12: a source pixel x with geometry (alpha >= 1/255) is un-projected at
// its surface depth z = depth / alpha (depth is the alpha-blended view z) and
// re-projected into the destination camera; V[x] = x' - x.  The operator w of
// Eq. 13 is a forward splat: x lands on the destination pixel containing x'
// (if x' is in front of the near plane), the nearest destination depth wins
// and ties go to the lower source index.  The warped gradient is the chain
// rule through the warp, (I + dV/dx)^-T times the source gradient, with dV/dx
// by central differences over source pixels with geometry (one-sided where a
// neighbour is missing, zero where both are).
//
// Everything that decides a landing pixel or a depth (z, the world point,
// the destination point, x') is FP64 in one fixed order of correctly rounded
// operations, contraction off, so both are reproducible bit for bit:
//   z = depth / alpha;  Xc = (((u - cx)/fx) z, ((v - cy)/fy) z, z)
//   Xw_i = (R0i (Xc0 - t0) + R1i (Xc1 - t1)) + R2i (Xc2 - t2)
//   Xd_i = ((R'i0 Xw0 + R'i1 Xw1) + R'i2 Xw2) + t'_i
//   u' = fx' (Xd0 / Xd2) + cx',  v' = fy' (Xd1 / Xd2) + cy'.
//
// Three launches: the z-buffer fill; the motion kernel (V in FP64, kept in
// the workspace for the resolve when gradients are warped, rounded to float32
// for the motion output, then a 64-bit atomic minimum of (float32 z' bits
// << 32 | source index) on the landing pixel, which is the depth test and the
// tie-break in one); and the resolve kernel (read the winner, copy its
// colour, emit its depth from the key's high word, and map its gradient
// through (I + dV/dx)^-T from the FP64 V of the winner and its four
// neighbours; a normal map, when given, is re-expressed in the destination
// camera's axes, R' R^T n, in a fixed FP64 order).  All three stream planar
// buffers and are HBM-bound.  One thread per pixel and a 1D grid whose
// blocks run in XCD-local runs of 64: the atomics of a wave fall on a few
// cache lines of one destination row, and the rows a block's neighbours touch
// mostly share its L2.
// (Four pixels per thread, 256 apart, measured no faster at 3840x2160 and
// slower at 960x540, where it leaves two waves per SIMD.)

#include "gs_kernels.hpp"

#pragma clang fp contract(off)

namespace gs {

namespace {

constexpr int kWarpThreads = 256;
constexpr double kWarpNear = 0.2;
constexpr unsigned long long kEmpty = ~0ull;
// workgroups per XCD run (measured at 960x540 and 3840x2160: 64 beats both
// the plain round-robin order and one contiguous range per XCD)
constexpr int64_t kWarpChunk = 64;

struct WarpPix {
    double ud, vd, zd;
    bool geom, ok;
};

// Eq. 12 for pixel (i, j) with alpha a and blended depth d, in the pinned order
__device__ __forceinline__ WarpPix motion_of(const WarpCams& c, float a, float d, int i, int j) {
    WarpPix p;
    p.geom = a >= kAlphaMin;
    // (the division is unconditional so the depth load is issued beside the
    // alpha load instead of after the geometry test)
    const double zq = (double)d / (p.geom ? (double)a : 1.0);
    const double z = p.geom ? zq : 1.0;
    const double U = (double)i + 0.5, Vv = (double)j + 0.5;
    const double xc0 = ((U - c.cxs) / c.fxs) * z;
    const double xc1 = ((Vv - c.cys) / c.fys) * z;
    const double e0 = xc0 - c.ts[0], e1 = xc1 - c.ts[1], e2 = z - c.ts[2];
    double xw[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) xw[k] = (c.Rs[k] * e0 + c.Rs[3 + k] * e1) + c.Rs[6 + k] * e2;
    double xd[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        xd[k] = ((c.Rd[3 * k] * xw[0] + c.Rd[3 * k + 1] * xw[1]) + c.Rd[3 * k + 2] * xw[2]) + c.td[k];
    p.zd = xd[2];
    p.ok = p.geom && p.zd >= kWarpNear;
    const double zs = p.ok ? p.zd : 1.0;
    p.ud = c.fxd * (xd[0] / zs) + c.cxd;
    p.vd = c.fyd * (xd[1] / zs) + c.cyd;
    return p;
}

__global__ void __launch_bounds__(kWarpThreads) k_zbuf_fill(ulonglong2* __restrict__ zbuf2, int64_t n2) {
    const int64_t e = (int64_t)blockIdx.x * kWarpThreads + threadIdx.x;
    if (e < n2) zbuf2[e] = make_ulonglong2(kEmpty, kEmpty);
}

// V of a pixel without geometry: a NaN pair (V itself is finite for finite inputs)
__device__ __forceinline__ bool has_geom(const double2& v) { return v.x == v.x; }

// one source pixel per thread, s = 256 b + threadIdx.x, b the block in
// XCD-run order
__global__ void __launch_bounds__(kWarpThreads) k_motion(WarpCams c, const float* __restrict__ alpha,
                                                         const float* __restrict__ depth,
                                                         float* __restrict__ motion, double2* __restrict__ vbuf,
                                                         unsigned long long* __restrict__ zbuf) {
    const int64_t HW = (int64_t)c.W * c.H;
    const int64_t s = xcd_chunked_block(blockIdx.x, gridDim.x, kWarpChunk) * kWarpThreads + threadIdx.x;
    if (s >= HW) return;
    // source index < 2^24: 32-bit division
    const uint32_t j = (uint32_t)s / (uint32_t)c.W, i = (uint32_t)s - j * (uint32_t)c.W;
    const WarpPix p = motion_of(c, alpha[s], depth[s], (int)i, (int)j);
    const double nan = __builtin_nan("");
    const double vx = p.geom ? p.ud - ((double)i + 0.5) : nan;
    const double vy = p.geom ? p.vd - ((double)j + 0.5) : nan;
    if (vbuf) vbuf[s] = make_double2(vx, vy);   // only the gradients' Jacobian reads it
    if (motion) {
        motion[s] = p.geom ? (float)vx : 0.0f;
        motion[HW + s] = p.geom ? (float)vy : 0.0f;
    }
    if (!p.ok) return;
    // the landing pixel; coordinates far outside are clamped first (no int overflow)
    const double cu = fmin(fmax(p.ud, -1.0), (double)c.Wd + 1.0);
    const double cv = fmin(fmax(p.vd, -1.0), (double)c.Hd + 1.0);
    const int ti = (int)floor(cu), tj = (int)floor(cv);
    if (ti < 0 || ti >= c.Wd || tj < 0 || tj >= c.Hd) return;
    const float zf = (float)p.zd;   // >= 0.2, so its bits order like its value
    const unsigned long long key = ((unsigned long long)__float_as_uint(zf) << 32) | (unsigned long long)s;
    atomicMin(&zbuf[(int64_t)tj * c.Wd + ti], key);
}

// dV/dx of source pixel s = j W + i from the FP64 motion plane: columns
// d/dx (neighbours s -/+ 1) and d/dy (s -/+ W), central where both
// neighbours have geometry, one-sided where one has, zero where none has
__device__ __forceinline__ void jacobian_at(const WarpCams& c, const double2* __restrict__ vbuf, uint32_t s,
                                            uint32_t i, uint32_t j, double Jm[2][2]) {
    const double2 v0 = vbuf[s];
#pragma unroll
    for (int axis = 0; axis < 2; ++axis) {
        const bool inp = axis == 0 ? i + 1 < (uint32_t)c.W : j + 1 < (uint32_t)c.H;
        const bool inm = axis == 0 ? i > 0 : j > 0;
        const uint32_t step = axis == 0 ? 1u : (uint32_t)c.W;
        const double2 vp = vbuf[inp ? s + step : s];
        const double2 vm = vbuf[inm ? s - step : s];
        const bool hp = inp && has_geom(vp), hm = inm && has_geom(vm);
        double dx, dy;
        if (hp && hm) {
            dx = (vp.x - vm.x) / 2.0;
            dy = (vp.y - vm.y) / 2.0;
        } else if (hp) {
            dx = vp.x - v0.x;
            dy = vp.y - v0.y;
        } else if (hm) {
            dx = v0.x - vm.x;
            dy = v0.y - vm.y;
        } else {
            dx = 0.0;
            dy = 0.0;
        }
        Jm[0][axis] = dx;
        Jm[1][axis] = dy;
    }
}

// one destination pixel per thread, k = 256 b + threadIdx.x, b the block in
// XCD-run order
__global__ void __launch_bounds__(kWarpThreads) k_warp_resolve(WarpCams c, const float* __restrict__ rgb,
                                                               const float* __restrict__ dcdx,
                                                               const float* __restrict__ dcdy,
                                                               const float* __restrict__ normal,
                                                               const double2* __restrict__ vbuf,
                                                               const unsigned long long* __restrict__ zbuf,
                                                               WarpOut o) {
    const int64_t HWd = (int64_t)c.Wd * c.Hd;
    const int64_t HW = (int64_t)c.W * c.H;
    const int64_t k = xcd_chunked_block(blockIdx.x, gridDim.x, kWarpChunk) * kWarpThreads + threadIdx.x;
    if (k >= HWd) return;
    const unsigned long long w = zbuf[k];
    if (w == kEmpty) {
        // a hole: nobody landed here
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            if (o.rgb) o.rgb[ch * HWd + k] = 0.0f;
            if (o.dcdx) o.dcdx[ch * HWd + k] = 0.0f;
            if (o.dcdy) o.dcdy[ch * HWd + k] = 0.0f;
            if (o.normal) o.normal[ch * HWd + k] = 0.0f;
        }
        if (o.depth) o.depth[k] = 0.0f;
        if (o.weight) o.weight[k] = 0.0f;
        if (o.source) o.source[k] = -1;
        return;
    }
    // source index < 2^24: 32-bit division.  Every input is read before the
    // first output is written (the output planes may not be assumed apart
    // from the inputs, so later loads could not move above the stores).
    const uint32_t s = (uint32_t)w;
    const bool grads = o.dcdx || o.dcdy;
    float col[3] = {0.f, 0.f, 0.f}, nrm[3] = {0.f, 0.f, 0.f}, gx[3] = {0.f, 0.f, 0.f}, gy[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        if (o.rgb) col[ch] = rgb[ch * HW + s];
        if (o.normal) nrm[ch] = normal[ch * HW + s];
        if (grads) {
            gx[ch] = dcdx[ch * HW + s];
            gy[ch] = dcdy[ch * HW + s];
        }
    }
    double Jm[2][2];
    if (grads) {
        const uint32_t j = s / (uint32_t)c.W, i = s - j * (uint32_t)c.W;
        jacobian_at(c, vbuf, s, i, j, Jm);
    }
    if (o.rgb) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) o.rgb[ch * HWd + k] = col[ch];
    }
    if (o.depth) o.depth[k] = __uint_as_float((uint32_t)(w >> 32));
    if (o.weight) o.weight[k] = 1.0f;
    if (o.source) o.source[k] = (int32_t)s;
    if (o.normal) {
        // source camera axes -> world ((R0i n0 + R1i n1) + R2i n2) -> destination axes
        const double n0 = nrm[0], n1 = nrm[1], n2 = nrm[2];
        double wv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) wv[a] = (c.Rs[a] * n0 + c.Rs[3 + a] * n1) + c.Rs[6 + a] * n2;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            o.normal[a * HWd + k] = (float)((c.Rd[3 * a] * wv[0] + c.Rd[3 * a + 1] * wv[1]) + c.Rd[3 * a + 2] * wv[2]);
    }
    if (!grads) return;
    // (I + J)^-T = [[d, -c], [-b, a]] / det for I + J = [[a, b], [c, d]]
    const double a = 1.0 + Jm[0][0], b = Jm[0][1], cc = Jm[1][0], d = 1.0 + Jm[1][1];
    const double det = a * d - b * cc;
    const double idet = det == 0.0 ? 0.0 : 1.0 / det;   // a fold of the motion field has no gradient
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        if (o.dcdx) o.dcdx[ch * HWd + k] = (float)((d * (double)gx[ch] - cc * (double)gy[ch]) * idet);
        if (o.dcdy) o.dcdy[ch * HWd + k] = (float)((a * (double)gy[ch] - b * (double)gx[ch]) * idet);
    }
}

}  // namespace

size_t warp_workspace_bytes(int64_t src_pixels, int64_t dst_pixels) {
    // z-buffer padded to 16 B, then the FP64 motion vectors
    return (size_t)((dst_pixels + 1) / 2) * 16 + (size_t)src_pixels * 16;
}

hipError_t launch_motion_warp(const WarpCams& c, const float* rgb, const float* alpha, const float* depth,
                              const float* dcdx, const float* dcdy, const float* normal, float* motion,
                              const WarpOut& o, void* workspace, hipStream_t st) {
    const int64_t HWd = (int64_t)c.Wd * c.Hd;
    const int64_t n2 = (HWd + 1) / 2;
    ulonglong2* zbuf2 = (ulonglong2*)workspace;
    double2* vbuf = (double2*)(zbuf2 + n2);
    unsigned long long* zbuf = (unsigned long long*)workspace;
    const bool grads = o.dcdx || o.dcdy;
    hipLaunchKernelGGL(k_zbuf_fill, dim3((unsigned)((n2 + kWarpThreads - 1) / kWarpThreads)), dim3(kWarpThreads), 0,
                       st, zbuf2, n2);
    const int64_t HW = (int64_t)c.W * c.H;
    hipLaunchKernelGGL(k_motion, dim3((unsigned)((HW + kWarpThreads - 1) / kWarpThreads)), dim3(kWarpThreads), 0, st,
                       c, alpha, depth, motion, grads ? vbuf : nullptr, zbuf);
    hipLaunchKernelGGL(k_warp_resolve, dim3((unsigned)((HWd + kWarpThreads - 1) / kWarpThreads)), dim3(kWarpThreads),
                       0, st, c, rgb, dcdx, dcdy, normal, (const double2*)vbuf, (const unsigned long long*)zbuf, o);
    return hipGetLastError();
}

}  // namespace gs
