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
// whole forward pass stays asynchronous and capturable).  The first launch
// also sets the n_zero words at `zero` to 0 (the frame's counters), which
// saves the frame a launch of its own.
__global__ void k_upload_jobs(JobChunk chunk, int count, JobDev* __restrict__ dst, uint32_t* __restrict__ zero,
                              int n_zero) {
    const int w = sizeof(JobDev) / 4;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(chunk.j);
    uint32_t* out = reinterpret_cast<uint32_t*>(dst);
    for (int i = threadIdx.x; i < count * w; i += blockDim.x) out[i] = src[i];
    for (int i = threadIdx.x; i < n_zero; i += blockDim.x) zero[i] = 0u;
}

hipError_t launch_upload_jobs(const JobDev* host_jobs, int n_jobs, JobDev* dev_jobs, hipStream_t st, uint32_t* zero,
                              int n_zero) {
    for (int b = 0; b < n_jobs; b += kUploadChunk) {
        JobChunk c;
        const int cnt = (n_jobs - b) < kUploadChunk ? (n_jobs - b) : kUploadChunk;
        for (int k = 0; k < cnt; ++k) c.j[k] = host_jobs[b + k];
        hipLaunchKernelGGL(k_upload_jobs, dim3(1), dim3(256), 0, st, c, cnt, dev_jobs + b, b == 0 ? zero : nullptr,
                           b == 0 ? n_zero : 0);
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

// A fill whose first thread also writes one job descriptor, passed as a
// kernel argument, to table[0]: a single frame's job upload without a launch
// of its own.
__global__ void k_fill_u32_job(uint32_t* __restrict__ p, uint32_t value, int64_t n, const JobDev one,
                               JobDev* __restrict__ table) {
    if (blockIdx.x == 0 && threadIdx.x == 0) table[0] = one;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

hipError_t launch_fill_u32_job(uint32_t* p, uint32_t value, int64_t n, const JobDev& one, JobDev* table,
                               hipStream_t st) {
    const int64_t blocks = n > 0 ? (n + 255) / 256 : 1;
    hipLaunchKernelGGL(k_fill_u32_job, dim3((unsigned)blocks), dim3(256), 0, st, p, value, n, one, table);
    return hipGetLastError();
}

// Pair emission in depth order.  Block b owns depth-sorted positions
// [256 b, 256 b + 256), whose pairs occupy a contiguous run of slots; its
// first slot is the sum of the chunk counts before it.  The block stages
// each Gaussian's first slot, rectangle origin and width in LDS, then fills
// the run window by window (2048 slots): each thread takes 8 consecutive
// slots (one binary search for the first, then a forward walk; positions
// without tiles share the next one's start and are skipped), stages the
// (tile, Gaussian) pairs in LDS, and the block writes the window out fully
// coalesced whatever the rectangle sizes.  Slots at or beyond `capacity`
// are dropped and flagged in counters[1].
// kExact (a frame of the batch uses the ellipse overlap mode): a position's
// tile count is the projection's.  Each ellipse-mode Gaussian of the block
// tabulates its box rows once (first slot and first column of each row,
// from ellipse_row_span on its record) in an LDS pool, and a slot finds its
// row by binary search there; Gaussians beyond the pool's room walk their
// rows instead, keeping the walk across a thread's consecutive slots.
constexpr int kEmitThreads = 256;
#ifndef GS_EMIT_PER
#define GS_EMIT_PER 4
#endif
constexpr int kEmitPer = GS_EMIT_PER;                    // slots per thread per window
constexpr int kEmitWin = kEmitThreads * kEmitPer;
constexpr int kEmitStride = kEmitPer + 1;                // padded LDS row: no bank conflicts
constexpr int kRowPool = 2048;                           // kExact: tabulated box rows per block
constexpr uint32_t kNoPool = 0xFFFFFFFFu;

// KeyT: uint16_t when the pairs are sorted by one pass (every tile id fits
// 11 bits), uint32_t for the two-pass sort of global tile ids.
template <bool kExact, typename KeyT>
__global__ void __launch_bounds__(kEmitThreads) k_emit(const JobDev* __restrict__ jobs, int n_jobs, int64_t n_flat,
                                                       const uint32_t* __restrict__ order,
                                                       const uint32_t* __restrict__ chunk_counts,
                                                       const uint32_t* __restrict__ depth_rects,
                                                       const uint32_t* __restrict__ touched,
                                                       const GaussRec* __restrict__ rec,
                                                       KeyT* __restrict__ tile_keys,
                                                       uint32_t* __restrict__ tile_vals, int64_t capacity,
                                                       uint32_t* __restrict__ counters) {
    __shared__ uint32_t s_off[kEmitThreads];
    __shared__ uint32_t s_g[kEmitThreads];
    __shared__ uint32_t s_row0[kEmitThreads];   // global tile id of the rectangle's top-left tile
    __shared__ uint32_t s_w[kEmitThreads];      // rectangle width in tiles
    __shared__ uint32_t s_tx[kEmitThreads];     // tiles per row of the frame
    __shared__ float s_inv[kEmitThreads];       // 1 / width
    __shared__ uint32_t s_key[kEmitThreads * kEmitStride];
    __shared__ uint32_t s_val[kEmitThreads * kEmitStride];
    __shared__ uint32_t s_red[kEmitThreads / 64 + 1];
    // kExact: the packed box of ellipse-mode Gaussians (kEmptyRect otherwise) and the frame's first tile id
    __shared__ uint32_t s_ebox[kExact ? kEmitThreads : 1];
    __shared__ uint32_t s_tb[kExact ? kEmitThreads : 1];
    // kExact: per tabulated row (first slot << 9 | first column), each Gaussian's first entry, wave row totals
    __shared__ uint32_t s_rows[kExact ? kRowPool : 1];
    __shared__ uint32_t s_pool[kExact ? kEmitThreads : 1];
    __shared__ uint32_t s_hred[kEmitThreads / 64];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t i = b * kEmitThreads + tid;
    const uint32_t* part = chunk_counts;
    const uint32_t* sup = chunk_counts + (n_flat + kChunk - 1) / kChunk;
    constexpr int kPerSup = kSuperChunk / kChunk;

    // every global read that does not depend on another is issued first
    // (unconditional loads from clamped indices, then a scheduling barrier:
    // a conditional load waits at the end of its branch, and the scheduler
    // would otherwise place each load next to its use)
    const int64_t sb = b / kPerSup;   // first slot of the block: whole 4096-position chunks,
    const int sj = (int)(b % kPerSup);   // then 256-position ones
    const int64_t ic = i < n_flat ? i : n_flat - 1;
    uint32_t r = depth_rects[ic];
    uint32_t g = order[ic];
    const uint32_t sup0 = sup[tid < sb ? tid : 0];
    const uint32_t part0 = part[sb * kPerSup + (tid < sj ? tid : 0)];
    __builtin_amdgcn_sched_barrier(0);
    if (i >= n_flat) {
        r = kEmptyRect;
        g = 0;
    }
    uint32_t pre = (tid < sb ? sup0 : 0u) + (tid < sj ? part0 : 0u);
    for (int64_t k = tid + kEmitThreads; k < sb; k += kEmitThreads) pre += sup[k];
    g = (int64_t)g < n_flat ? g : 0u;
    const int jg = n_jobs == 1 ? 0 : find_job_gauss(jobs, n_jobs, (int64_t)g);
    const uint32_t txn = (uint32_t)jobs[jg].tiles_x;
    const uint32_t tbase = (uint32_t)jobs[jg].tile_base;
    const bool ell = kExact && jobs[jg].overlap == kOverlapEllipse;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) pre += (uint32_t)__shfl_xor((int)pre, o, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = pre;

    const uint32_t v = kExact ? (i < n_flat ? touched[g] : 0u) : rect_tiles(r);
    // inclusive scan of the block's tile counts (and, kExact, of the box
    // rows that ellipse-mode Gaussians tabulate)
    const uint32_t hrows = (ell && v) ? (r >> 24) - ((r >> 8) & 0xFFu) + 1u : 0u;
    uint32_t inc = v, hinc = hrows;
    const int lane = tid & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)inc, o, 64);
        if (lane >= o) inc += t;
        if (kExact) {
            const uint32_t th = (uint32_t)__shfl_up((int)hinc, o, 64);
            if (lane >= o) hinc += th;
        }
    }
    __syncthreads();
    if (lane == 63) {
        s_off[tid >> 6] = inc;   // wave totals, briefly
        s_hred[tid >> 6] = hinc;
    }
    __syncthreads();
    uint32_t base = 0, start = 0, tot = 0, hbase = 0;
#pragma unroll
    for (int w = 0; w < kEmitThreads / 64; ++w) {
        start += s_red[w];
        const uint32_t wt = s_off[w];
        base += w < (tid >> 6) ? wt : 0u;
        tot += wt;
        if (kExact) hbase += w < (tid >> 6) ? s_hred[w] : 0u;
    }
    hbase += hinc - hrows;
    __syncthreads();
    s_off[tid] = start + base + inc - v;
    const uint32_t end = start + tot;
    if (i < n_flat) {
        const uint32_t rx0 = r & 0xFFu, ry0 = (r >> 8) & 0xFFu, rx1 = (r >> 16) & 0xFFu;
        s_g[tid] = g;
        s_row0[tid] = tbase + ry0 * txn + rx0;
        const uint32_t w = v ? rx1 - rx0 + 1u : 1u;
        s_w[tid] = w;
        s_inv[tid] = 1.0f / (float)w;
        s_tx[tid] = txn;
        if (kExact) {
            s_ebox[tid] = ell ? r : kEmptyRect;
            s_tb[tid] = tbase;
            s_pool[tid] = kNoPool;
            if (hrows && hbase + hrows <= (uint32_t)kRowPool) {
                const GaussRec rr = rec[g];
                const EllipseCover e0 = ellipse_cover(rr.u, rr.v, rr.A, rr.B, rr.C, rr.o);
                const int bx0 = (int)(r & 0xFFu), by0 = (int)((r >> 8) & 0xFFu), bx1 = (int)((r >> 16) & 0xFFu);
                uint32_t first = 0;
                for (uint32_t k = 0; k < hrows; ++k) {
                    int c0, c1;
                    ellipse_row_span(e0, by0 + (int)k, bx0, bx1, c0, c1);
                    s_rows[hbase + k] = (first << 9) | (uint32_t)c0;
                    first += c1 >= c0 ? (uint32_t)(c1 - c0 + 1) : 0u;
                }
                s_pool[tid] = hbase;
            }
        }
    }
    __syncthreads();

    // kExact: the walk of this thread's current ellipse-mode Gaussian
    int cur = -1, cur_ty = 0, cur_c0 = 0, cur_bx0 = 0, cur_bx1 = 0, cur_by1 = 0;
    uint32_t cur_start = 0, cur_w = 0;
    EllipseCover ec = {};

    bool over = false;
    int lo = 0;
    for (uint32_t w0 = start; w0 < end; w0 += kEmitWin) {
        const uint32_t s0 = w0 + (uint32_t)(tid * kEmitPer);
        if (s0 < end) {
            int hi = kEmitThreads - 1;   // slots only grow, so the previous position bounds the search
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= s0) lo = mid; else hi = mid - 1;
            }
#pragma unroll
            for (int k = 0; k < kEmitPer; ++k) {
                const uint32_t slot = s0 + k;
                if (slot < end) {
                    while (lo + 1 < kEmitThreads && s_off[lo + 1] <= slot) ++lo;
                    const uint32_t local = slot - s_off[lo];
                    if (kExact && s_ebox[lo] != kEmptyRect && s_pool[lo] != kNoPool) {
                        // the tabulated row holding this slot: the last whose first slot is <= local
                        const uint32_t p0 = s_pool[lo], bx = s_ebox[lo];
                        const int by0 = (int)((bx >> 8) & 0xFFu);
                        int a = 0, z = (int)(bx >> 24) - by0;
                        while (a < z) {
                            const int mid = (a + z + 1) >> 1;
                            if ((s_rows[p0 + mid] >> 9) <= local) a = mid; else z = mid - 1;
                        }
                        const uint32_t e = s_rows[p0 + a];
                        s_key[tid * kEmitStride + k] = s_tb[lo] + (uint32_t)(by0 + a) * s_tx[lo] +
                                                       ((e & 0x1FFu) + (local - (e >> 9)));
                        s_val[tid * kEmitStride + k] = s_g[lo];
                        continue;
                    }
                    if (kExact && s_ebox[lo] != kEmptyRect) {
                        if (lo != cur) {
                            // a new Gaussian: its cover, and its first row
                            cur = lo;
                            const GaussRec rr = rec[s_g[lo]];
                            ec = ellipse_cover(rr.u, rr.v, rr.A, rr.B, rr.C, rr.o);
                            const uint32_t bx = s_ebox[lo];
                            cur_bx0 = (int)(bx & 0xFFu);
                            cur_ty = (int)((bx >> 8) & 0xFFu);
                            cur_bx1 = (int)((bx >> 16) & 0xFFu);
                            cur_by1 = (int)(bx >> 24);
                            int c1;
                            ellipse_row_span(ec, cur_ty, cur_bx0, cur_bx1, cur_c0, c1);
                            cur_start = 0u;
                            cur_w = c1 >= cur_c0 ? (uint32_t)(c1 - cur_c0 + 1) : 0u;
                        }
                        // rows only advance: slots of one Gaussian come in order
                        while (local >= cur_start + cur_w && cur_ty < cur_by1) {
                            cur_start += cur_w;
                            ++cur_ty;
                            int c1;
                            ellipse_row_span(ec, cur_ty, cur_bx0, cur_bx1, cur_c0, c1);
                            cur_w = c1 >= cur_c0 ? (uint32_t)(c1 - cur_c0 + 1) : 0u;
                        }
                        s_key[tid * kEmitStride + k] = s_tb[lo] + (uint32_t)cur_ty * s_tx[lo] +
                                                       (uint32_t)(cur_c0 + (int)(local - cur_start));
                        s_val[tid * kEmitStride + k] = s_g[lo];
                        continue;
                    }
                    const uint32_t w = s_w[lo];
                    // row = local / w from a float estimate, corrected to the exact quotient
                    int ty = (int)(((float)local + 0.5f) * s_inv[lo]);
                    int tx = (int)local - ty * (int)w;
                    if (tx >= (int)w) { ++ty; tx -= (int)w; }
                    if (tx < 0) { --ty; tx += (int)w; }
                    s_key[tid * kEmitStride + k] = s_row0[lo] + (uint32_t)ty * s_tx[lo] + (uint32_t)tx;
                    s_val[tid * kEmitStride + k] = s_g[lo];
                }
            }
        }
        __syncthreads();
        const uint32_t nwin = (end - w0) < (uint32_t)kEmitWin ? (end - w0) : (uint32_t)kEmitWin;
        for (uint32_t q = tid; q < nwin; q += kEmitThreads) {
            const uint32_t slot = w0 + q;
            const uint32_t li = (q / kEmitPer) * kEmitStride + q % kEmitPer;
            if ((int64_t)slot < capacity) {
                tile_keys[slot] = (KeyT)s_key[li];
                tile_vals[slot] = s_val[li];
            } else {
                over = true;
            }
        }
        __syncthreads();
    }
    if (over) counters[1] = 1u;
}

hipError_t launch_emit(const JobDev* jobs, int n_jobs, int64_t n_flat, const uint32_t* order,
                       const uint32_t* chunk_counts, const uint32_t* depth_rects, const uint32_t* touched,
                       const GaussRec* rec, void* tile_keys, bool narrow_keys, uint32_t* tile_vals, int64_t capacity,
                       uint32_t* counters, hipStream_t st) {
    if (n_flat == 0) return hipSuccess;
    const dim3 grid((unsigned)((n_flat + kEmitThreads - 1) / kEmitThreads));
#define GS_EMIT(EXACT, KT)                                                                                       \
    hipLaunchKernelGGL((k_emit<EXACT, KT>), grid, dim3(kEmitThreads), 0, st, jobs, n_jobs, n_flat, order,         \
                       chunk_counts, depth_rects, touched, rec, static_cast<KT*>(tile_keys), tile_vals, capacity, \
                       counters)
    if (touched && narrow_keys)
        GS_EMIT(true, uint16_t);
    else if (touched)
        GS_EMIT(true, uint32_t);
    else if (narrow_keys)
        GS_EMIT(false, uint16_t);
    else
        GS_EMIT(false, uint32_t);
#undef GS_EMIT
    return hipGetLastError();
}

// Banded emission (a batch over 2048 tiles, no ellipse overlap).  Band b's
// pairs fill one run, after the runs of bands 0..b-1, in depth order and,
// per Gaussian, rows then columns of its rectangle's rows inside the band;
// the key is the tile id local to the band.  Workgroup (x, b) owns the same
// 256 depth positions as block x of k_emit, and only their pairs in band b:
// its first position in the band's run comes from the band's chunk counts
// (the exclusive prefix of the 4096-position counts, then the 256-position
// counts before it), and it fills its part window by window as k_emit does,
// so every window is written out as one contiguous run.  A workgroup whose
// positions have no pair in its band ends at once.  (Walking all bands'
// pairs of a block once and splitting each window by band at write-out was
// measured slower: its writes scatter over the bands' runs.)
__global__ void __launch_bounds__(kEmitThreads) k_emit_banded(const JobDev* __restrict__ jobs, int n_jobs,
                                                              int64_t n_flat, const uint32_t* __restrict__ order,
                                                              const uint32_t* __restrict__ chunk_counts,
                                                              const uint32_t* __restrict__ depth_rects, int nb,
                                                              const uint32_t* __restrict__ band_cnt,
                                                              uint16_t* __restrict__ tile_keys,
                                                              uint32_t* __restrict__ tile_vals, int64_t capacity,
                                                              uint32_t* __restrict__ counters) {
    __shared__ int64_t s_off[kEmitThreads];
    __shared__ uint32_t s_g[kEmitThreads];
    __shared__ uint32_t s_row0[kEmitThreads];   // band-local tile id of the clipped rectangle's top-left tile
    __shared__ uint32_t s_w[kEmitThreads];
    __shared__ uint32_t s_tx[kEmitThreads];
    __shared__ float s_inv[kEmitThreads];
    __shared__ uint32_t s_key[kEmitThreads * kEmitStride];
    __shared__ uint32_t s_val[kEmitThreads * kEmitStride];
    __shared__ uint32_t s_wt[kEmitThreads / 64];
    __shared__ uint32_t s_term[kEmitThreads / 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int64_t b = blockIdx.x;
    const int band = blockIdx.y;
    const int64_t i = b * kEmitThreads + tid;
    const int64_t words = chunk_count_words(n_flat);
    const int64_t nchunk = (n_flat + kChunk - 1) / kChunk;
    constexpr int kPerSup = kSuperChunk / kChunk;
    const int64_t sb = b / kPerSup;
    const int sj = (int)(b % kPerSup);
    const uint32_t* part = chunk_counts + band * words;
    const uint32_t tot = part[b];   // this workgroup's pairs
    if (tot == 0) return;

    // first position: the run start of the band (the pairs of the bands
    // before it: lanes 0..band-1 of wavefront 0), the band's pairs of the
    // 4096-position chunks before this block (one prefix word), then of its
    // 256-position chunks (lanes 0..sj-1 of wavefront 1); the terms are
    // summed with the scan's barrier below.  All loads unconditional from
    // clamped indices, issued before any use.
    const int64_t ic = i < n_flat ? i : n_flat - 1;
    uint32_t r = depth_rects[ic];
    uint32_t g = order[ic];
    const uint32_t tb = band_cnt[lane < band ? lane : 0];
    const uint32_t tp = part[sb * kPerSup + (lane < sj ? lane : 0)];
    const uint32_t pre_sup = part[nchunk + sb];
    __builtin_amdgcn_sched_barrier(0);
    if (i >= n_flat) {
        r = kEmptyRect;
        g = 0;
    }
    uint32_t term = 0;
    if ((tid >> 6) == 0) term = lane < band ? tb : 0u;
    if ((tid >> 6) == 1) term = lane < sj ? tp : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) term += (uint32_t)__shfl_xor((int)term, o, 64);
    g = (int64_t)g < n_flat ? g : 0u;
    const int jg = n_jobs == 1 ? 0 : find_job_gauss(jobs, n_jobs, (int64_t)g);
    const uint32_t txn = (uint32_t)jobs[jg].tiles_x;
    const uint32_t tbase = (uint32_t)jobs[jg].tile_base;
    const int R = jobs[jg].band_rows, B0 = jobs[jg].band0, nbj = (jobs[jg].tiles_y + R - 1) / R;
    const uint32_t bt0 = (uint32_t)jobs[jg].band_tile0;
    // this position's rows inside the band
    const int kb = band - B0;
    int rlo = 0, rhi = -1, w = 1;
    if (i < n_flat && kb >= 0 && kb < nbj) band_rect(r, kb, R, rlo, rhi, w);
    const uint32_t v = rhi >= rlo ? (uint32_t)((rhi - rlo + 1) * w) : 0u;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) s_wt[tid >> 6] = inc;
    if (lane == 0) s_term[tid >> 6] = term;
    __syncthreads();
    uint32_t wbase = 0;
    int64_t start = (int64_t)pre_sup;
#pragma unroll
    for (int w2 = 0; w2 < kEmitThreads / 64; ++w2) {
        wbase += w2 < (tid >> 6) ? s_wt[w2] : 0u;
        start += s_term[w2];
    }
    const int64_t end = start + tot;
    s_off[tid] = start + wbase + inc - v;
    if (i < n_flat && v) {
        s_g[tid] = g;
        s_tx[tid] = txn;
        s_row0[tid] = tbase + (uint32_t)rlo * txn + (r & 0xFFu) - (bt0 + (uint32_t)(kb * R) * txn);
        s_w[tid] = (uint32_t)w;
        s_inv[tid] = 1.0f / (float)w;
    }
    __syncthreads();

    bool over = end > capacity;   // pairs at or beyond the capacity are dropped
    int lo = 0;
    for (int64_t w0 = start; w0 < end && w0 < capacity; w0 += kEmitWin) {
        const int64_t s0 = w0 + tid * kEmitPer;
        if (s0 < end) {
            int hi = kEmitThreads - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= s0) lo = mid; else hi = mid - 1;
            }
#pragma unroll
            for (int k = 0; k < kEmitPer; ++k) {
                const int64_t slot = s0 + k;
                if (slot < end) {
                    while (lo + 1 < kEmitThreads && s_off[lo + 1] <= slot) ++lo;
                    const uint32_t local = (uint32_t)(slot - s_off[lo]);
                    const uint32_t ww = s_w[lo];
                    int ty = (int)(((float)local + 0.5f) * s_inv[lo]);
                    int tx = (int)local - ty * (int)ww;
                    if (tx >= (int)ww) { ++ty; tx -= (int)ww; }
                    if (tx < 0) { --ty; tx += (int)ww; }
                    s_key[tid * kEmitStride + k] = s_row0[lo] + (uint32_t)ty * s_tx[lo] + (uint32_t)tx;
                    s_val[tid * kEmitStride + k] = s_g[lo];
                }
            }
        }
        __syncthreads();
        const int64_t nwin = (end - w0) < kEmitWin ? (end - w0) : kEmitWin;
        for (int64_t q = tid; q < nwin; q += kEmitThreads) {
            const int64_t slot = w0 + q;
            const int64_t li = (q / kEmitPer) * kEmitStride + q % kEmitPer;
            if (slot < capacity) {
                tile_keys[slot] = (uint16_t)s_key[li];
                tile_vals[slot] = s_val[li];
            } else {
                over = true;
            }
        }
        __syncthreads();
    }
    if (over) counters[1] = 1u;
}

hipError_t launch_emit_banded(const JobDev* jobs, int n_jobs, int64_t n_flat, const uint32_t* order,
                              const uint32_t* chunk_counts, const uint32_t* depth_rects, int nb,
                              const uint32_t* band_cnt, uint16_t* tile_keys, uint32_t* tile_vals, int64_t capacity,
                              uint32_t* counters, hipStream_t st) {
    if (n_flat == 0) return hipSuccess;
    if (nb < 1 || nb > kMaxBands) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n_flat + kEmitThreads - 1) / kEmitThreads), (unsigned)nb);
    hipLaunchKernelGGL(k_emit_banded, grid, dim3(kEmitThreads), 0, st, jobs, n_jobs, n_flat, order, chunk_counts,
                       depth_rects, nb, band_cnt, tile_keys, tile_vals, capacity, counters);
    return hipGetLastError();
}

// Tile list boundaries of the sorted tile ids: four consecutive elements per
// thread (one 16-byte load plus the neighbours on either side).
__global__ void __launch_bounds__(256) k_ranges(const uint32_t* __restrict__ st, DevCount n,
                                                uint32_t* __restrict__ ranges, int64_t n_tiles) {
    int64_t cnt = n.cap;
    if (n.dev_count) {
        const int64_t c = (int64_t)*n.dev_count;
        cnt = c < n.cap ? c : n.cap;
    }
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= cnt) return;
    uint32_t v[6];
    v[0] = i0 > 0 ? st[i0 - 1] : 0xFFFFFFFFu;
    if (i0 + 4 <= cnt) {
        const uint4 q = *reinterpret_cast<const uint4*>(st + i0);
        v[1] = q.x; v[2] = q.y; v[3] = q.z; v[4] = q.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[1 + k] = (i0 + k < cnt) ? st[i0 + k] : 0xFFFFFFFFu;
    }
    v[5] = (i0 + 4 < cnt) ? st[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = i0 + k;
        if (i >= cnt) break;
        const uint32_t t = v[1 + k];
        if ((int64_t)t >= n_tiles) continue;
        if (v[k] != t) ranges[2 * (int64_t)t] = (uint32_t)i;
        if (v[k + 2] != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
    }
}

hipError_t launch_ranges(const uint32_t* sorted_tiles, DevCount n, uint32_t* ranges, int64_t n_tiles,
                         hipStream_t st) {
    hipError_t e = launch_fill_u32(ranges, 0u, 2 * n_tiles, st);
    if (e != hipSuccess) return e;
    if (n.cap == 0) return hipSuccess;
    const int64_t threads = (n.cap + 3) / 4;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, sorted_tiles, n, ranges,
                       n_tiles);
    return hipGetLastError();
}

// 64-bit (local tile << 32 | depth key) keys of one job's sorted pairs, from
// its tiles' ranges: one workgroup per tile writes that tile's run.
__global__ void __launch_bounds__(256) k_compose_keys(const uint32_t* __restrict__ ranges,
                                                      const uint32_t* __restrict__ sv,
                                                      const uint32_t* __restrict__ zkey, int64_t begin,
                                                      int64_t gauss_base, uint64_t* __restrict__ keys_out,
                                                      uint32_t* __restrict__ vals_out) {
    const int64_t t = blockIdx.x;
    const uint32_t r0 = ranges[2 * t], r1 = ranges[2 * t + 1];
    for (int64_t i = (int64_t)r0 + threadIdx.x; i < (int64_t)r1; i += blockDim.x) {
        const uint32_t g = sv[i];
        keys_out[i - begin] = ((uint64_t)t << 32) | (uint64_t)zkey[g];
        vals_out[i - begin] = (uint32_t)((int64_t)g - gauss_base);
    }
}

hipError_t launch_compose_keys(const uint32_t* job_ranges, int64_t tiles, const uint32_t* sorted_vals,
                               const uint32_t* zkey, int64_t begin, int64_t gauss_base, uint64_t* keys_out,
                               uint32_t* vals_out, hipStream_t st) {
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compose_keys, dim3((unsigned)tiles), dim3(256), 0, st, job_ranges, sorted_vals, zkey, begin,
                       gauss_base, keys_out, vals_out);
    return hipGetLastError();
}

}  // namespace gs
