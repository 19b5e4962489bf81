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
// tile overlap modes (the values of GS_OVERLAP_SQUARE / GS_OVERLAP_OPACITY)
constexpr int kOverlapSquare = 0;
constexpr int kOverlapOpacity = 1;

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
    int32_t overlap;        // kOverlapSquare or kOverlapOpacity
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

}  // namespace gs
