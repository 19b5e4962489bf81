// Shared device-side definitions of the gfx950 rasterizer: the per-frame job
// descriptor the kernels read from device memory, the per-Gaussian record
// the projection writes for compositing, and the rasterizer's constants.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

// Constants of the method (3DGS^3 Sec. 3 builds on the 3DGS rasterizer; the
// thresholds are its conventions, float32 values nearest 1/255, 1e-4, 0.99).
constexpr int kTile = 16;
constexpr double kGuard = 1.3;
constexpr double kSigmaCut = 3.0;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kColorOffset = 0.5f;
constexpr int kMaxJobs = 64;
constexpr uint32_t kCulledKey = 0xFFFFFFFFu;
// tile overlap modes (the values of GS_OVERLAP_SQUARE / _OPACITY / _ELLIPSE)
constexpr int kOverlapSquare = 0;
constexpr int kOverlapOpacity = 1;
constexpr int kOverlapEllipse = 2;

// Flat Gaussian ranges are padded to multiples of this so a projection block
// never straddles two frames.
constexpr int kGaussAlign = 256;

struct alignas(16) JobDev {
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* opac;
    const float* sh;
    int64_t n;
    int64_t gauss_base;     // first flat Gaussian index of the frame
    int32_t sh_degree;
    int32_t tile_base;      // first global tile id of the frame
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    double R[9];
    double t[3];
    double fx, fy, cx, cy;
    double near_z, dilation;
    float bg[3];
    int32_t overlap;        // kOverlapSquare, kOverlapOpacity or kOverlapEllipse
    // tile bands of a batch over 2048 tiles: the frame's first band, the tile
    // rows per band (tiles_y when the frame shares one band with other
    // frames) and the global id of the first tile of its first band; band k
    // of the frame starts at band_tile0 + k * band_rows * tiles_x
    int32_t band0, band_rows, band_tile0;
    float* rgb;
    float* alpha;
    float* depth;
    float* dcdx;
    float* dcdy;
    float* final_T;
    uint32_t* n_contrib;
    uint32_t* n_evaluated;
    uint32_t* n_blended;
    float* normal;
    float* nv;
};

// What compositing needs of one projected Gaussian: the 2D mean in FP64 (so a
// tile-relative float offset can be formed exactly), the conic (inverse 2D
// covariance), opacity, colour and view z.
struct alignas(16) GaussRec {
    double u, v;
    float A, B, C, o;
    float r, g, b, z;
};
static_assert(sizeof(GaussRec) == 48, "record layout");

// Index of the frame owning flat index `i` given the ascending bases.
__device__ __forceinline__ int find_job_gauss(const JobDev* jobs, int n_jobs, int64_t i) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].gauss_base <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// MI355X dispatches consecutive workgroups round-robin to its 8 XCDs, each
// with its own L2.  Workgroup b of nblk takes logical block
// x * (nblk / 8) + min(x, nblk % 8) + b / 8 (x = b % 8), so that every XCD
// works through one contiguous logical range and neighbouring blocks, which
// read overlapping lines, share an L2.
constexpr int kXcdCount = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblk) {
    const int64_t q = nblk / kXcdCount, r = nblk % kXcdCount;
    const int64_t x = b % kXcdCount;
    return x * q + (x < r ? x : r) + b / kXcdCount;
}

// The same idea for long streaming grids: rounds of 8 x chunk workgroups, in
// which XCD x takes chunk consecutive logical blocks, so the XCDs sweep the
// data side by side while each keeps runs of neighbouring blocks (the last,
// partial round keeps the identity order).
__device__ __forceinline__ int64_t xcd_chunked_block(int64_t b, int64_t nblk, int64_t chunk) {
    const int64_t round = kXcdCount * chunk;
    const int64_t g = b / round;
    if ((g + 1) * round > nblk) return b;
    const int64_t r = b - g * round;
    return g * round + (r % kXcdCount) * chunk + r / kXcdCount;
}

__device__ __forceinline__ int find_job_tile(const JobDev* jobs, int n_jobs, int64_t t) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The alpha' >= 1/255 ellipse of one Gaussian, as the tile-overlap test of
// kOverlapEllipse sees it: mean (u, v) in pixels and the stored float32
// conic (A, B, C) and opacity o of its record, so that the projection (which
// counts the tiles) and the emission (which lists them) decide alike (the
// same float32 operations, never contracted, on the same values).  The
// ellipse is q(d) = A dx^2 + 2 B dx dy + C dy^2 <= Qm, d = pixel - mean,
// Qm = 2 ln(255 o) with the compositing cull's margins (0.1 % + 1e-3); its
// half-widths are xe = sqrt(Qm C / det), ye = sqrt(Qm A / det).  Conics with
// B^2 > 0.996 A C keep every tile of their box (full).
struct EllipseCover {
    float u, v, A, B, iA, det, AQ, xe, ye, yr, mx, my;
    bool full;
};

__device__ __forceinline__ EllipseCover ellipse_cover(double u, double v, float A, float B, float C, float o) {
#pragma clang fp contract(off)
    EllipseCover e;
    e.u = (float)u;
    e.v = (float)v;
    e.A = A;
    e.B = B;
    e.det = A * C - B * B;
    // 2 ln(255 o) = 2 ln 2 (log2 o - log2(1/255))
    const float Q = 1.3862943611198906f * (__log2f(o) + 7.994353436858858f);
    const float Qm = (Q > 0.f ? Q : 0.f) * 1.001f + 1e-3f;
    e.full = !(A > 0.f) || !(C > 0.f) || !(e.det > 4e-3f * (A * C));
    const float qd = e.full ? 0.f : Qm / e.det;
    e.xe = __builtin_sqrtf(qd * C);
    e.ye = __builtin_sqrtf(qd * A);
    e.iA = e.full ? 0.f : 1.f / A;
    e.AQ = A * Qm;
    e.yr = e.full ? 0.f : (B * e.xe) / C;   // the chord's right end peaks at dy = -yr, its left end at dy = yr
    e.mx = 0.001f * e.xe + 0.02f;
    e.my = 0.001f * e.ye + 0.02f;
    return e;
}

// Tile columns [c0, c1] of tile row ty (within the box columns [bx0, bx1])
// whose pixel centres the ellipse can reach; c0 > c1 when it reaches none.
// The row's pixel centres span dy in [16 ty + 0.5 - v, 16 ty + 15.5 - v],
// widened by 0.1 % of ye + 0.02 px and clipped to [-ye, ye].  Over that band
// the right end of the ellipse's chord, (-B dy + sqrt(A Qm - det dy^2)) / A,
// is concave in dy with its maximum at dy = -B xe / C, so its largest value
// is taken there or at the band end nearest to it; the left end likewise
// (minimum at dy = B xe / C).  Both ends are widened by 0.1 % of xe + 0.02
// px (far above the float32 rounding of these few operations), and a tile
// column is kept when its pixel centres meet [u + left, u + right].
__device__ __forceinline__ void ellipse_row_span(const EllipseCover& e, int ty, int bx0, int bx1, int& c0,
                                                 int& c1) {
#pragma clang fp contract(off)
    if (e.full) {
        c0 = bx0;
        c1 = bx1;
        return;
    }
    const float y0 = (float)(kTile * ty);
    float lo = ((y0 + 0.5f) - e.v) - e.my;
    float hi = ((y0 + 15.5f) - e.v) + e.my;
    lo = lo > -e.ye ? lo : -e.ye;
    hi = hi < e.ye ? hi : e.ye;
    if (lo > hi) {
        c0 = 1;
        c1 = 0;
        return;
    }
    const float yr = -e.yr < lo ? lo : (-e.yr > hi ? hi : -e.yr);
    const float yl = e.yr < lo ? lo : (e.yr > hi ? hi : e.yr);
    const float sr = e.AQ - e.det * (yr * yr);
    const float sl = e.AQ - e.det * (yl * yl);
    const float right = (__builtin_sqrtf(sr > 0.f ? sr : 0.f) - e.B * yr) * e.iA + e.mx;
    const float left = (-__builtin_sqrtf(sl > 0.f ? sl : 0.f) - e.B * yl) * e.iA - e.mx;
    const float a = __builtin_ceilf(((e.u + left) - 15.5f) * (1.f / (float)kTile));
    const float b = __builtin_floorf(((e.u + right) - 0.5f) * (1.f / (float)kTile));
    // (clamped in float first: a far-off ellipse must not overflow the conversion)
    c0 = a > (float)bx0 ? (a < (float)(bx1 + 1) ? (int)a : bx1 + 1) : bx0;
    c1 = b < (float)bx1 ? (b > (float)(bx0 - 1) ? (int)b : bx0 - 1) : bx1;
}

}  // namespace gs
