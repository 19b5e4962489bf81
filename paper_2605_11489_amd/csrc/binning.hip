// Binning kernels: job-table upload, (tile, Gaussian) pair emission in depth
// order, per-tile list ranges, and composition of the 64-bit
// (tile << 32 | depth bits) keys for inspection.
#include "gs_kernels.hpp"

namespace gs {

namespace {
constexpr int kUploadChunk = 8;
struct JobChunk {
    JobDev j[kUploadChunk];
};
}  // namespace

// Job descriptors travel as kernel arguments (no host staging buffer, so the
// whole forward pass stays asynchronous and capturable).
__global__ void k_upload_jobs(JobChunk chunk, int count, JobDev* __restrict__ dst) {
    const int w = sizeof(JobDev) / 4;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(chunk.j);
    uint32_t* out = reinterpret_cast<uint32_t*>(dst);
    for (int i = threadIdx.x; i < count * w; i += blockDim.x) out[i] = src[i];
}

hipError_t launch_upload_jobs(const JobDev* host_jobs, int n_jobs, JobDev* dev_jobs, hipStream_t st) {
    for (int b = 0; b < n_jobs; b += kUploadChunk) {
        JobChunk c;
        const int cnt = (n_jobs - b) < kUploadChunk ? (n_jobs - b) : kUploadChunk;
        for (int k = 0; k < cnt; ++k) c.j[k] = host_jobs[b + k];
        hipLaunchKernelGGL(k_upload_jobs, dim3(1), dim3(256), 0, st, c, cnt, dev_jobs + b);
    }
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, value, n);
    return hipGetLastError();
}

// One thread per depth-sorted Gaussian: its covered tiles, row by row, get
// consecutive slots starting at the exclusive scan of tile counts.  Slots at
// or beyond `capacity` are dropped and flagged in counters[1].
__global__ void __launch_bounds__(256) k_emit(const JobDev* __restrict__ jobs, int n_jobs, int64_t n_flat,
                                              const uint32_t* __restrict__ order, const uint32_t* __restrict__ offsets,
                                              const ushort4* __restrict__ rect, const uint32_t* __restrict__ touched,
                                              uint32_t* __restrict__ tile_keys,
                                              uint32_t* __restrict__ tile_vals, int64_t capacity,
                                              uint32_t* __restrict__ counters) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_flat) return;
    const uint32_t g = order[i];
    if ((int64_t)g >= n_flat || touched[g] == 0u) return;   // culled or off-screen: no tiles
    const ushort4 r = rect[g];
    const int w = (int)r.z - (int)r.x + 1;
    const int h = (int)r.w - (int)r.y + 1;
    const int j = find_job_gauss(jobs, n_jobs, (int64_t)g);
    const int tx_n = jobs[j].tiles_x;
    const uint32_t tb = (uint32_t)jobs[j].tile_base;
    int64_t slot = offsets[i];
    bool over = false;
    for (int ty = 0; ty < h; ++ty) {
        const uint32_t row = tb + (uint32_t)((r.y + ty) * tx_n + r.x);
        for (int tx = 0; tx < w; ++tx, ++slot) {
            if (slot < capacity) {
                tile_keys[slot] = row + (uint32_t)tx;
                tile_vals[slot] = g;
            } else {
                over = true;
            }
        }
    }
    if (over) counters[1] = 1u;
}

hipError_t launch_emit(const JobDev* jobs, int n_jobs, int64_t n_flat, const uint32_t* order,
                       const uint32_t* offsets, const ushort4* rect, const uint32_t* touched, uint32_t* tile_keys,
                       uint32_t* tile_vals, int64_t capacity, uint32_t* counters, hipStream_t st) {
    if (n_flat == 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)((n_flat + 255) / 256)), dim3(256), 0, st, jobs, n_jobs, n_flat,
                       order, offsets, rect, touched, tile_keys, tile_vals, capacity, counters);
    return hipGetLastError();
}

__global__ void k_ranges(const uint32_t* __restrict__ st, DevCount n, uint32_t* __restrict__ ranges,
                         int64_t n_tiles) {
    int64_t cnt = n.cap;
    if (n.dev_count) {
        const int64_t c = (int64_t)*n.dev_count;
        cnt = c < n.cap ? c : n.cap;
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const uint32_t t = st[i];
    if ((int64_t)t >= n_tiles) return;
    if (i == 0 || st[i - 1] != t) ranges[2 * (int64_t)t] = (uint32_t)i;
    if (i == cnt - 1 || st[i + 1] != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
}

hipError_t launch_ranges(const uint32_t* sorted_tiles, DevCount n, uint32_t* ranges, int64_t n_tiles,
                         hipStream_t st) {
    hipError_t e = launch_fill_u32(ranges, 0u, 2 * n_tiles, st);
    if (e != hipSuccess) return e;
    if (n.cap == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((n.cap + 255) / 256)), dim3(256), 0, st, sorted_tiles, n, ranges, n_tiles);
    return hipGetLastError();
}

__global__ void k_compose_keys(const uint32_t* __restrict__ st, const uint32_t* __restrict__ sv,
                               const uint32_t* __restrict__ zkey, int64_t begin, int64_t count, int64_t tile_base,
                               int64_t gauss_base, uint64_t* __restrict__ keys_out,
                               uint32_t* __restrict__ vals_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t g = sv[begin + i];
    keys_out[i] = ((uint64_t)(st[begin + i] - (uint32_t)tile_base) << 32) | (uint64_t)zkey[g];
    vals_out[i] = (uint32_t)((int64_t)g - gauss_base);
}

hipError_t launch_compose_keys(const uint32_t* sorted_tiles, const uint32_t* sorted_vals, const uint32_t* zkey,
                               int64_t begin, int64_t count, int64_t tile_base, int64_t gauss_base,
                               uint64_t* keys_out, uint32_t* vals_out, hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compose_keys, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, sorted_tiles,
                       sorted_vals, zkey, begin, count, tile_base, gauss_base, keys_out, vals_out);
    return hipGetLastError();
}

}  // namespace gs
