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
// Three launches: the z-buffer fill, the motion kernel (one thread per source
// pixel: V, then a 64-bit atomic minimum of (float32 z' bits << 32 | source
// index) on the landing pixel, which is the depth test and the tie-break in
// one), and the resolve kernel (one thread per destination pixel: read the
// winner, copy its colour, emit its depth from the key's high word, and map
// its gradient through (I + dV/dx)^-T, recomputing V at the four neighbours
// in FP64 rather than storing it).  All three stream planar float32 buffers
// and are HBM-bound.
#include "gs_kernels.hpp"

#pragma clang fp contract(off)

namespace gs {

namespace {

constexpr int kWarpThreads = 256;
constexpr double kWarpNear = 0.2;
constexpr unsigned long long kEmpty = ~0ull;

struct WarpPix {
    double ud, vd, zd;
    bool geom, ok;
};

__device__ __forceinline__ WarpPix motion_at(const WarpCams& c, const float* __restrict__ alpha,
                                             const float* __restrict__ depth, int i, int j) {
    WarpPix p;
    const int64_t s = (int64_t)j * c.W + i;
    const float a = alpha[s];
    p.geom = a >= kAlphaMin;
    const double z = p.geom ? (double)depth[s] / (double)a : 1.0;
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

__global__ void __launch_bounds__(kWarpThreads) k_zbuf_fill(unsigned long long* __restrict__ zbuf, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * kWarpThreads + threadIdx.x;
    if (e < n) zbuf[e] = kEmpty;
}

__global__ void __launch_bounds__(kWarpThreads) k_motion(WarpCams c, const float* __restrict__ alpha,
                                                         const float* __restrict__ depth,
                                                         float* __restrict__ motion,
                                                         unsigned long long* __restrict__ zbuf) {
    const int64_t HW = (int64_t)c.W * c.H;
    const int64_t s = (int64_t)blockIdx.x * kWarpThreads + threadIdx.x;
    if (s >= HW) return;
    const int j = (int)(s / c.W), i = (int)(s - (int64_t)j * c.W);
    const WarpPix p = motion_at(c, alpha, depth, i, j);
    if (motion) {
        motion[s] = p.geom ? (float)(p.ud - ((double)i + 0.5)) : 0.0f;
        motion[HW + s] = p.geom ? (float)(p.vd - ((double)j + 0.5)) : 0.0f;
    }
    if (!p.ok) return;
    // the landing pixel; coordinates far outside are clamped first (no int overflow)
    const double cu = fmin(fmax(p.ud, -1.0), (double)c.Wd + 1.0);
    const double cv = fmin(fmax(p.vd, -1.0), (double)c.Hd + 1.0);
    const int ti = (int)floor(cu), tj = (int)floor(cv);
    if (ti < 0 || ti >= c.Wd || tj < 0 || tj >= c.Hd) return;
    const float zf = (float)p.zd;   // >= 0.2, so its bit pattern orders like its value
    const unsigned long long key = ((unsigned long long)__float_as_uint(zf) << 32) | (unsigned long long)s;
    atomicMin(&zbuf[(int64_t)tj * c.Wd + ti], key);
}

// (V at (i, j)) for a pixel with geometry
__device__ __forceinline__ void motion_vec(const WarpPix& p, int i, int j, double& vx, double& vy) {
    vx = p.ud - ((double)i + 0.5);
    vy = p.vd - ((double)j + 0.5);
}

__global__ void __launch_bounds__(kWarpThreads) k_warp_resolve(WarpCams c, const float* __restrict__ rgb,
                                                               const float* __restrict__ alpha,
                                                               const float* __restrict__ depth,
                                                               const float* __restrict__ dcdx,
                                                               const float* __restrict__ dcdy,
                                                               const unsigned long long* __restrict__ zbuf,
                                                               WarpOut o) {
    const int64_t HWd = (int64_t)c.Wd * c.Hd;
    const int64_t HW = (int64_t)c.W * c.H;
    const int64_t k = (int64_t)blockIdx.x * kWarpThreads + threadIdx.x;
    if (k >= HWd) return;
    const unsigned long long w = zbuf[k];
    if (w == kEmpty) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            if (o.rgb) o.rgb[ch * HWd + k] = 0.0f;
            if (o.dcdx) o.dcdx[ch * HWd + k] = 0.0f;
            if (o.dcdy) o.dcdy[ch * HWd + k] = 0.0f;
        }
        if (o.depth) o.depth[k] = 0.0f;
        if (o.weight) o.weight[k] = 0.0f;
        if (o.source) o.source[k] = -1;
        return;
    }
    const int64_t s = (int64_t)(uint32_t)w;
    const int j = (int)(s / c.W), i = (int)(s - (int64_t)j * c.W);
    if (o.rgb) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) o.rgb[ch * HWd + k] = rgb[ch * HW + s];
    }
    if (o.depth) o.depth[k] = __uint_as_float((uint32_t)(w >> 32));
    if (o.weight) o.weight[k] = 1.0f;
    if (o.source) o.source[k] = (int32_t)s;
    if (!o.dcdx && !o.dcdy) return;
    // dV/dx: columns d/dx (neighbours i -/+ 1) and d/dy (j -/+ 1)
    double vx0, vy0;
    motion_vec(motion_at(c, alpha, depth, i, j), i, j, vx0, vy0);
    double Jm[2][2];
#pragma unroll
    for (int axis = 0; axis < 2; ++axis) {
        const int di = axis == 0 ? 1 : 0, dj = axis == 0 ? 0 : 1;
        const int ip = i + di, jp = j + dj, im = i - di, jm = j - dj;
        double pvx = 0.0, pvy = 0.0, mvx = 0.0, mvy = 0.0;
        bool hp = ip < c.W && jp < c.H, hm = im >= 0 && jm >= 0;
        if (hp) {
            const WarpPix q = motion_at(c, alpha, depth, ip, jp);
            hp = q.geom;
            motion_vec(q, ip, jp, pvx, pvy);
        }
        if (hm) {
            const WarpPix q = motion_at(c, alpha, depth, im, jm);
            hm = q.geom;
            motion_vec(q, im, jm, mvx, mvy);
        }
        double dx, dy;
        if (hp && hm) {
            dx = (pvx - mvx) / 2.0;
            dy = (pvy - mvy) / 2.0;
        } else if (hp) {
            dx = pvx - vx0;
            dy = pvy - vy0;
        } else if (hm) {
            dx = vx0 - mvx;
            dy = vy0 - mvy;
        } else {
            dx = 0.0;
            dy = 0.0;
        }
        Jm[0][axis] = dx;
        Jm[1][axis] = dy;
    }
    // (I + J)^-T = [[d, -c], [-b, a]] / det for I + J = [[a, b], [c, d]]
    const double a = 1.0 + Jm[0][0], b = Jm[0][1], cc = Jm[1][0], d = 1.0 + Jm[1][1];
    const double det = a * d - b * cc;
    const bool fold = det == 0.0;   // the motion field folds: no gradient is defined
    const double idet = fold ? 0.0 : 1.0 / det;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const double gx = dcdx[ch * HW + s], gy = dcdy[ch * HW + s];
        if (o.dcdx) o.dcdx[ch * HWd + k] = (float)((d * gx - cc * gy) * idet);
        if (o.dcdy) o.dcdy[ch * HWd + k] = (float)((a * gy - b * gx) * idet);
    }
}

}  // namespace

hipError_t launch_motion_warp(const WarpCams& c, const float* rgb, const float* alpha, const float* depth,
                              const float* dcdx, const float* dcdy, float* motion, const WarpOut& o,
                              unsigned long long* zbuf, hipStream_t st) {
    const int64_t HW = (int64_t)c.W * c.H, HWd = (int64_t)c.Wd * c.Hd;
    const unsigned gd = (unsigned)((HWd + kWarpThreads - 1) / kWarpThreads);
    const unsigned gs = (unsigned)((HW + kWarpThreads - 1) / kWarpThreads);
    hipLaunchKernelGGL(k_zbuf_fill, dim3(gd), dim3(kWarpThreads), 0, st, zbuf, HWd);
    hipLaunchKernelGGL(k_motion, dim3(gs), dim3(kWarpThreads), 0, st, c, alpha, depth, motion, zbuf);
    hipLaunchKernelGGL(k_warp_resolve, dim3(gd), dim3(kWarpThreads), 0, st, c, rgb, alpha, depth, dcdx, dcdy,
                       (const unsigned long long*)zbuf, o);
    return hipGetLastError();
}

}  // namespace gs
