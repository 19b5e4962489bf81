// Direct binning: the (tile, Gaussian) pairs of one frame are written
// straight into their per-tile depth order, without a sort over the pairs.
//
// The per-tile lists are depth-sorted (3DGS^3 Sec. 3): list t holds, in
// depth order, every Gaussian whose tile rectangle contains t.  With the
// Gaussians already in depth order (the depth sort), the list position of
// the pair (t, g) is the number of pairs of tile t before it:
//   pos(t, g) = start[t] + #{g' before g in depth order : t in rect(g')}.
// The depth order is cut into chunks of 256 positions, and the count splits
// into the pairs of tile t in earlier chunks (a per-chunk, per-tile count
// matrix and its prefix over the chunks: k_bin_count, k_bin_group,
// k_bin_gscan) and the pairs of tile t among the earlier Gaussians of the
// same chunk.  The latter comes from coverage masks: for each wavefront of
// 64 Gaussians, one 64-bit ballot per tile column (whose rectangles span the
// column) and one per tile row, so that the Gaussians covering tile (x, y)
// are mx[x] & my[y] and the earlier ones a popcount away (k_bin_emit).
// A rectangle is the only shape this handles, so frames with the exact
// ellipse overlap take the sorted path, and so do batches of several frames
// (their depth order interleaves the frames' Gaussians).
//
// Work per pair: one 4-byte scattered write and a few LDS reads; per chunk
// and tile: 2 B written by the count and read twice by the prefix passes, and
// the emission stages its chunk's row of list offsets (4 B per tile).
#include "gs_kernels.hpp"

namespace gs {

namespace {

constexpr int kBinThreads = 256;
constexpr int kBinWaves = kBinThreads / 64;
constexpr int kBinGroup = 16;          // chunks per group of the prefix over chunks
constexpr int kBinPer = 4;             // pairs per thread per window of the enumeration
constexpr int kBinWin = kBinThreads * kBinPer;

// Exclusive block-wide scan of one value per thread (256 threads); `red`
// holds kBinWaves + 1 words.  Returns the exclusive prefix, sets total.
__device__ __forceinline__ uint32_t bin_block_scan(uint32_t v, uint32_t* red, uint32_t& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) red[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kBinWaves; ++w) {
        const uint32_t s = red[w];
        before += w < wave ? s : 0u;
        all += s;
    }
    __syncthreads();
    total = all;
    return before + inc - v;
}

// Row and column (inside the rectangle, row major, width w, 1/w
// precomputed) of the local-th pair of a rectangle: the row from a float
// estimate corrected to the exact quotient.
__device__ __forceinline__ void rect_pair_rc(uint32_t local, uint32_t w, float inv_w, int& ty, int& tx) {
    ty = (int)(((float)local + 0.5f) * inv_w);
    tx = (int)local - ty * (int)w;
    if (tx >= (int)w) { ++ty; tx -= (int)w; }
    if (tx < 0) { --ty; tx += (int)w; }
}

}  // namespace

// Per chunk of 256 depth positions, the number of pairs of every tile
// (u16, at most 256), one row of tpad entries per chunk.  LDS: one u32
// counter per tile (dynamic, 4 T bytes).
__global__ void __launch_bounds__(kBinThreads) k_bin_count(const uint32_t* __restrict__ depth_rects, int64_t n_flat,
                                                           int tiles_x, int n_tiles, int tpad,
                                                           uint16_t* __restrict__ hist) {
    extern __shared__ uint32_t cnt[];
    __shared__ uint32_t s_off[kBinThreads];
    __shared__ uint32_t s_row0[kBinThreads];
    __shared__ uint32_t s_w[kBinThreads];
    __shared__ float s_inv[kBinThreads];
    __shared__ uint32_t red[kBinWaves + 1];
    const int tid = threadIdx.x;
    const int64_t chunk = blockIdx.x;
    const int64_t i = chunk * kBinThreads + tid;
    const uint32_t r = i < n_flat ? depth_rects[i] : kEmptyRect;
    for (int t = tid; t < n_tiles; t += kBinThreads) cnt[t] = 0u;
    const uint32_t v = rect_tiles(r);
    uint32_t total;
    const uint32_t off = bin_block_scan(v, red, total);
    s_off[tid] = off;
    const uint32_t w = v ? ((r >> 16) & 0xFFu) - (r & 0xFFu) + 1u : 1u;
    s_w[tid] = w;
    s_inv[tid] = 1.0f / (float)w;
    s_row0[tid] = ((r >> 8) & 0xFFu) * (uint32_t)tiles_x + (r & 0xFFu);
    __syncthreads();
    int lo = 0;
    for (uint32_t w0 = 0; w0 < total; w0 += kBinWin) {
        const uint32_t s0 = w0 + (uint32_t)(tid * kBinPer);
        if (s0 < total) {
            int hi = kBinThreads - 1;   // slots only grow: the previous owner bounds the search
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= s0) lo = mid; else hi = mid - 1;
            }
#pragma unroll
            for (int k = 0; k < kBinPer; ++k) {
                const uint32_t slot = s0 + k;
                if (slot < total) {
                    while (lo + 1 < kBinThreads && s_off[lo + 1] <= slot) ++lo;
                    int ty, tx;
                    rect_pair_rc(slot - s_off[lo], s_w[lo], s_inv[lo], ty, tx);
                    atomicAdd(&cnt[s_row0[lo] + (uint32_t)ty * (uint32_t)tiles_x + (uint32_t)tx], 1u);
                }
            }
        }
    }
    __syncthreads();
    uint16_t* row = hist + chunk * tpad;
    for (int t = tid; t < tpad; t += kBinThreads) row[t] = t < n_tiles ? (uint16_t)cnt[t] : (uint16_t)0;
}

// Chunks in groups of 16: per tile, the counts of the group's chunks become
// their exclusive prefix inside the group (in place; at most 15 x 256, so
// still u16) and the group total goes to gsum[g][t].  Grid (groups,
// tpad / 256).
__global__ void __launch_bounds__(kBinThreads) k_bin_group(uint16_t* __restrict__ hist, uint32_t* __restrict__ gsum,
                                                           int64_t n_chunks, int tpad) {
    const int64_t g = blockIdx.x;
    const int t = blockIdx.y * kBinThreads + threadIdx.x;
    if (t >= tpad) return;
    uint32_t v[kBinGroup];
#pragma unroll
    for (int j = 0; j < kBinGroup; ++j) {
        const int64_t c = g * kBinGroup + j;
        v[j] = c < n_chunks ? hist[c * tpad + t] : 0u;
    }
    uint32_t run = 0;
#pragma unroll
    for (int j = 0; j < kBinGroup; ++j) {
        const int64_t c = g * kBinGroup + j;
        if (c < n_chunks) hist[c * tpad + t] = (uint16_t)run;
        run += v[j];
    }
    gsum[g * tpad + t] = run;
}

// Per tile, the exclusive prefix of the group totals over the groups (in
// place) and the tile's pair total.  A workgroup takes 64 tiles (one per
// lane) and splits the groups into 16 contiguous segments, one per wave.
constexpr int kBinSegs = 16;

__global__ void __launch_bounds__(64 * kBinSegs) k_bin_gscan(uint32_t* __restrict__ gsum,
                                                             uint32_t* __restrict__ totals, int64_t n_groups,
                                                             int tpad, uint32_t* __restrict__ pair_total) {
    __shared__ uint32_t part[kBinSegs][64];
    const int tl = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + tl;
    const bool own = t < tpad;
    const int64_t len = (n_groups + kBinSegs - 1) / kBinSegs;
    const int64_t g0 = seg * len;
    const int64_t g1 = (g0 + len < n_groups) ? g0 + len : n_groups;
    uint32_t sum = 0;
    if (own)
        for (int64_t g = g0; g < g1; ++g) sum += gsum[g * tpad + t];
    part[seg][tl] = sum;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kBinSegs; ++k) {
        const uint32_t v = part[k][tl];
        pre += k < seg ? v : 0u;
        tot += v;
    }
    if (own) {
        uint32_t run = pre;
        for (int64_t c0 = g0; c0 < g1; c0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = c0 + k < g1 ? gsum[(c0 + k) * tpad + t] : 0u;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (c0 + k < g1) gsum[(c0 + k) * tpad + t] = run;
                run += v[k];
            }
        }
        if (seg == 0) totals[t] = tot;
    }
    // the frame's pair count: one atomic per workgroup of 64 tiles
    if (seg == 0) {
        uint32_t w = own ? tot : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) w += (uint32_t)__shfl_xor((int)w, o, 64);
        if (tl == 0 && w) atomicAdd(pair_total, w);
    }
}

// Tile starts: the exclusive scan of the tile totals, in place, and the tile
// ranges [start, start + total) clamped to the capacity ([0, 0) for an
// empty tile).  One workgroup of 1024 threads, at most 8 tiles each.
constexpr int kStartThreads = 1024;

__global__ void __launch_bounds__(kStartThreads) k_bin_starts(uint32_t* __restrict__ totals, int n_tiles,
                                                              uint32_t* __restrict__ ranges, int64_t capacity) {
    __shared__ uint32_t red[kStartThreads / 64];
    constexpr int kPer = kDirectMaxTiles / kStartThreads;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int t0 = tid * kPer;
    uint32_t v[kPer];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        v[k] = t0 + k < n_tiles ? totals[t0 + k] : 0u;
        sum += v[k];
    }
    uint32_t inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) red[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += red[w];
    uint32_t run = before + inc - sum;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int t = t0 + k;
        if (t < n_tiles) {
            totals[t] = run;
            const uint64_t e = (uint64_t)run + v[k];
            const uint32_t a = (uint64_t)run < (uint64_t)capacity ? run : (uint32_t)capacity;
            const uint32_t b = e < (uint64_t)capacity ? (uint32_t)e : (uint32_t)capacity;
            reinterpret_cast<uint2*>(ranges)[t] = v[k] ? make_uint2(a, b) : make_uint2(0u, 0u);
            run += v[k];
        }
    }
}

// The pairs of one chunk written at their list positions.  Every block
// stages its chunk's list offset of every tile in LDS, builds the coverage
// masks of its four wavefronts, and enumerates its pairs in depth order.
// Positions at or beyond the capacity are dropped and flagged.  Dynamic
// LDS: 4 T bytes of offsets.
__global__ void __launch_bounds__(kBinThreads) k_bin_emit(const uint32_t* __restrict__ depth_rects,
                                                          const uint32_t* __restrict__ order, int64_t n_flat,
                                                          int tiles_x, int tiles_y, int tpad,
                                                          const uint16_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ gsum,
                                                          const uint32_t* __restrict__ starts,
                                                          uint32_t* __restrict__ tile_vals, int64_t capacity,
                                                          uint32_t* __restrict__ counters) {
    extern __shared__ uint32_t base[];
    __shared__ uint64_t mx[kBinWaves][256];
    __shared__ uint64_t my[kBinWaves][256];
    __shared__ uint32_t s_off[kBinThreads];
    __shared__ uint32_t s_row0[kBinThreads];
    __shared__ uint32_t s_w[kBinThreads];
    __shared__ float s_inv[kBinThreads];
    __shared__ uint32_t s_g[kBinThreads];
    __shared__ uint32_t red[kBinWaves + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // each XCD takes a contiguous run of chunks, so the consecutive list
    // positions that neighbouring chunks write meet in one L2
    const int64_t chunk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t grp = chunk / kBinGroup;
    const int n_tiles = tiles_x * tiles_y;
    const int64_t i = chunk * kBinThreads + tid;
    uint32_t r = kEmptyRect, g = 0;
    if (i < n_flat) {
        r = depth_rects[i];
        g = order[i];
    }

    // list offset of every tile for this chunk: its start, plus its pairs in
    // the earlier groups and in the earlier chunks of this group
    for (int t = tid; t < n_tiles; t += kBinThreads)
        base[t] = starts[t] + gsum[grp * tpad + t] + (uint32_t)hist[chunk * tpad + t];

    // coverage masks of this wavefront's 64 rectangles: bit `lane` of
    // mx[wave][x] (my[wave][y]) is set when the lane's rectangle spans
    // tile column x (row y); each lane sets its bits over its own columns
    // and rows with LDS atomics (cleared first)
    const bool has = rect_tiles(r) != 0u;
    const int rx0 = (int)(r & 0xFFu), ry0 = (int)((r >> 8) & 0xFFu), rx1 = (int)((r >> 16) & 0xFFu),
              ry1 = (int)(r >> 24);
    for (int x = lane; x < tiles_x; x += 64) mx[wave][x] = 0ull;
    for (int y = lane; y < tiles_y; y += 64) my[wave][y] = 0ull;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (has) {
        const uint64_t bit = 1ull << lane;
        for (int x = rx0; x <= rx1; ++x) atomicOr(&mx[wave][x], bit);
        for (int y = ry0; y <= ry1; ++y) atomicOr(&my[wave][y], bit);
    }

    // the chunk's pairs in depth order (Gaussians, then row-major tiles)
    const uint32_t v = rect_tiles(r);
    uint32_t total;
    const uint32_t off = bin_block_scan(v, red, total);   // (its barriers also publish base[] and the masks)
    s_off[tid] = off;
    const uint32_t w = v ? (uint32_t)(rx1 - rx0 + 1) : 1u;
    s_w[tid] = w;
    s_inv[tid] = 1.0f / (float)w;
    s_row0[tid] = ((uint32_t)ry0 << 16) | (uint32_t)rx0;
    s_g[tid] = g;
    __syncthreads();
    bool over = false;
    int lo = 0;
    for (uint32_t w0 = 0; w0 < total; w0 += kBinWin) {
        const uint32_t s0 = w0 + (uint32_t)(tid * kBinPer);
        if (s0 < total) {
            int hi = kBinThreads - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= s0) lo = mid; else hi = mid - 1;
            }
#pragma unroll
            for (int k = 0; k < kBinPer; ++k) {
                const uint32_t slot = s0 + k;
                if (slot < total) {
                    while (lo + 1 < kBinThreads && s_off[lo + 1] <= slot) ++lo;
                    int ry, rx;
                    rect_pair_rc(slot - s_off[lo], s_w[lo], s_inv[lo], ry, rx);
                    const uint32_t org = s_row0[lo];   // (top row << 16) | left column
                    const int ty = (int)(org >> 16) + ry, tx = (int)(org & 0xFFFFu) + rx;
                    const uint32_t t = (uint32_t)ty * (uint32_t)tiles_x + (uint32_t)tx;
                    const int ow = lo >> 6, ol = lo & 63;
                    // earlier Gaussians of the chunk covering tile t
                    uint32_t rank = (uint32_t)__popcll(mx[ow][tx] & my[ow][ty] & ((1ull << ol) - 1ull));
                    for (int q = 0; q < ow; ++q) rank += (uint32_t)__popcll(mx[q][tx] & my[q][ty]);
                    const uint64_t pos = (uint64_t)base[t] + rank;
                    if (pos < (uint64_t)capacity)
                        tile_vals[pos] = s_g[lo];
                    else
                        over = true;
                }
            }
        }
    }
    if (over) counters[1] = 1u;
}

static_assert(kDirectMaxTiles % kBinThreads == 0, "tile limit");

int64_t direct_bin_tpad(int64_t n_tiles) {
    int64_t p = 1;
    while (p < n_tiles) p <<= 1;
    return p < kBinThreads ? kBinThreads : p;
}

int64_t direct_bin_bytes(int64_t n_flat, int64_t n_tiles) {
    const int64_t chunks = (n_flat + kBinThreads - 1) / kBinThreads;
    const int64_t groups = (chunks + kBinGroup - 1) / kBinGroup;
    const int64_t tp = direct_bin_tpad(n_tiles);
    return ((chunks * tp * 2 + 255) / 256) * 256 + ((groups * tp * 4 + 255) / 256) * 256 + tp * 4;
}

namespace {
struct BinRegions {
    uint16_t* hist;
    uint32_t* gsum;
    uint32_t* totals;
    int64_t tpad, chunks, groups;
};

BinRegions bin_regions(void* scratch, int64_t n_flat, int64_t n_tiles) {
    BinRegions b;
    b.tpad = direct_bin_tpad(n_tiles);
    b.chunks = (n_flat + kBinThreads - 1) / kBinThreads;
    b.groups = (b.chunks + kBinGroup - 1) / kBinGroup;
    char* base = static_cast<char*>(scratch);
    b.hist = reinterpret_cast<uint16_t*>(base);
    base += ((b.chunks * b.tpad * 2 + 255) / 256) * 256;
    b.gsum = reinterpret_cast<uint32_t*>(base);
    base += ((b.groups * b.tpad * 4 + 255) / 256) * 256;
    b.totals = reinterpret_cast<uint32_t*>(base);
    return b;
}
}  // namespace

hipError_t launch_bin_count(const uint32_t* depth_rects, int64_t n_flat, int tiles_x, int tiles_y, void* scratch,
                            uint32_t* pair_total, hipStream_t st) {
    if (n_flat == 0) return hipSuccess;
    const int64_t n_tiles = (int64_t)tiles_x * tiles_y;
    const BinRegions b = bin_regions(scratch, n_flat, n_tiles);
    hipLaunchKernelGGL(k_bin_count, dim3((unsigned)b.chunks), dim3(kBinThreads), (size_t)n_tiles * 4, st,
                       depth_rects, n_flat, tiles_x, (int)n_tiles, (int)b.tpad, b.hist);
    hipLaunchKernelGGL(k_bin_group, dim3((unsigned)b.groups, (unsigned)(b.tpad / kBinThreads)), dim3(kBinThreads), 0,
                       st, b.hist, b.gsum, b.chunks, (int)b.tpad);
    hipLaunchKernelGGL(k_bin_gscan, dim3((unsigned)((b.tpad + 63) / 64)), dim3(64 * kBinSegs), 0, st, b.gsum,
                       b.totals, b.groups, (int)b.tpad, pair_total);
    return hipGetLastError();
}


hipError_t launch_bin_emit(const uint32_t* depth_rects, const uint32_t* order, int64_t n_flat, int tiles_x,
                           int tiles_y, void* scratch, uint32_t* ranges, uint32_t* tile_vals, int64_t capacity,
                           uint32_t* counters, hipStream_t st) {
    const int64_t n_tiles = (int64_t)tiles_x * tiles_y;
    if (n_flat == 0) return launch_fill_u32(ranges, 0u, 2 * n_tiles, st);
    const BinRegions b = bin_regions(scratch, n_flat, n_tiles);
    hipLaunchKernelGGL(k_bin_starts, dim3(1), dim3(kStartThreads), 0, st, b.totals, (int)n_tiles, ranges, capacity);
    hipLaunchKernelGGL(k_bin_emit, dim3((unsigned)b.chunks), dim3(kBinThreads), (size_t)n_tiles * 4, st,
                       depth_rects, order, n_flat, tiles_x, tiles_y, (int)b.tpad, b.hist, b.gsum, b.totals, tile_vals,
                       capacity, counters);
    return hipGetLastError();
}

}  // namespace gs
