// Launchers of the gfx950 kernels (internal to the library).
#pragma once

#include "gs_common.hpp"

namespace gs {

// Element count read on the device: min(*dev_count, cap) when dev_count is
// non-null, else cap.
struct DevCount {
    const uint32_t* dev_count;
    int64_t cap;
};

constexpr int kRsMaxBits = 11;                // digit bits per radix pass
constexpr int kRsMaxBins = 1 << kRsMaxBits;

// Blocks of one radix pass over at most `cap` elements (4096 per block), and
// the histogram scratch bytes a pass over them needs (16-bit counts per block
// and digit, 32-bit counts per group of 16 blocks and digit).
int64_t rs_pass_blocks(int64_t cap);
int64_t rs_hist_bytes(int64_t cap);
hipError_t launch_upload_jobs(const JobDev* host_jobs, int n_jobs, JobDev* dev_jobs, hipStream_t st,
                              uint32_t* zero = nullptr, int n_zero = 0);

// Packed tile rectangle: bytes (tx0, ty0, tx1, ty1) from low to high; an
// empty rectangle is kEmptyRect (tx1 < tx0).
constexpr uint32_t kEmptyRect = 0x000000FFu;
__host__ __device__ inline uint32_t rect_tiles(uint32_t r) {
    const int x0 = r & 0xFF, y0 = (r >> 8) & 0xFF, x1 = (r >> 16) & 0xFF, y1 = r >> 24;
    return (x1 >= x0 && y1 >= y0) ? (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1)) : 0u;
}

// Tile rows [lo, hi] of packed rectangle r inside band k of a frame cut
// into bands of R tile rows (hi < lo: none), and the rectangle's width.
__device__ __forceinline__ void band_rect(uint32_t r, int k, int R, int& lo, int& hi, int& w) {
    const int x0 = r & 0xFF, y0 = (r >> 8) & 0xFF, x1 = (r >> 16) & 0xFF, y1 = r >> 24;
    const int b0 = k * R, b1 = b0 + R - 1;
    lo = y0 > b0 ? y0 : b0;
    hi = y1 < b1 ? y1 : b1;
    w = x1 - x0 + 1;
    if (w <= 0 || y1 < y0) hi = lo - 1;
}

// nrm: per flat Gaussian (nx, ny, nz, 0), the camera-facing shortest-axis
// normal, written when non-null.
hipError_t launch_project(const JobDev* jobs, int n_jobs, int64_t n_flat, GaussRec* rec, uint32_t* zkey,
                          uint32_t* rect, uint32_t* touched, float4* nrm, hipStream_t st);
// A single frame: its descriptor goes as a kernel argument, and the first
// workgroup writes it to table[0] and clears zero[0, n_zero) (no upload
// launch before it).
hipError_t launch_project_one(const JobDev& one, JobDev* table, uint32_t* zero, int n_zero, int64_t n_flat,
                              GaussRec* rec, uint32_t* zkey, uint32_t* rect, uint32_t* touched, float4* nrm,
                              hipStream_t st);

// One stable LSD pass over `bits` (<= 11) bits starting at `shift` of
// (key, value) pairs.  vals_in == nullptr means values are the element
// indices; keys_out may be nullptr (values only).  vals2_in / vals2_out (both
// null or both set) add a second value that moves with its element: the
// element at position i lands at p with vals2_out[p] = vals2_in[i].
// ranges != nullptr (only with shift 0, when the digit is the whole tile id):
// also writes ranges[t] = [first, last + 1) of digit t, or [0, 0), for
// t < n_ranges <= 2^bits.
// Scratch: hist of rs_hist_bytes(cap) bytes (256-byte aligned) and totals [2^bits].
hipError_t radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, const uint32_t* vals2_in,
                      uint32_t* keys_out, uint32_t* vals_out, uint32_t* vals2_out, DevCount n, int shift, int bits,
                      void* hist, uint32_t* totals, uint32_t* ranges, int64_t n_ranges, hipStream_t st);

// Banded tile sort (a batch over 2048 tiles).  The global tile ids are cut
// into at most kMaxBands bands of at most 2048 consecutive tiles: whole
// frames packed together, or the tile rows of one large frame.  The emission
// writes each band's pairs as one contiguous run, in band order, with tile
// ids local to the band, so a single stable pass of at most 11 bits per band
// gives the global (tile, depth, index) order.
constexpr int kMaxBands = 64;
struct BandDesc {
    const uint32_t* cnt;            // per-band pair counts, on the device (filled by the chunk counts)
    int64_t cap;                    // key capacity: pairs beyond it are dropped
    int32_t nb;                     // bands
    uint32_t tile0[kMaxBands];      // first global tile id of each band
    uint32_t ntiles[kMaxBands];     // tiles of each band
};

// Stable pass over the bands' runs: keys are band-local tile ids (< 2^bits),
// values are written to vals_out at the same run positions, and each band's
// tile ranges (global positions) to ranges.  Scratch: seg_hist_bytes(cap, nb)
// bytes of histograms and nb x 2048 totals.
int64_t seg_hist_bytes(int64_t cap, int nb);
hipError_t radix_pass_banded(const uint16_t* keys_in, const uint32_t* vals_in, uint32_t* vals_out,
                             const BandDesc& bands, int bits, void* hist, uint32_t* totals, uint32_t* ranges,
                             hipStream_t st);

// The one-pass tile sort: 16-bit tile ids (< 2^bits) and their values;
// writes the sorted values and the tile ranges (n_ranges <= 2^bits tiles).
// The key buffer must hold three keys beyond the count.
hipError_t radix_pass_tiles(const uint16_t* keys_in, const uint32_t* vals_in, uint32_t* vals_out, DevCount n,
                            int bits, void* hist, uint32_t* totals, uint32_t* ranges, int64_t n_ranges,
                            hipStream_t st);

// Tile counts of depth-order chunks of kChunk and kSuperChunk positions
// (rect_tiles of the depth-sorted rectangles, or with `touched` non-null the
// projection's tile counts gathered through the depth order, which the
// ellipse overlap mode needs): counts holds chunk_count_words(n) words, the
// kChunk counts first, then the kSuperChunk counts; the total is added to
// *total (zeroed by the caller).
constexpr int kChunk = 256;
constexpr int kSuperChunk = 4096;
__host__ __device__ inline int64_t chunk_count_words(int64_t n) {
    return (n + kChunk - 1) / kChunk + (n + kSuperChunk - 1) / kSuperChunk + 2;
}
hipError_t launch_chunk_counts(const uint32_t* rects, const uint32_t* order, const uint32_t* touched, int64_t n,
                               uint32_t* counts, uint32_t* total, hipStream_t st);
// Banded: the counts of each of the nb bands (nb x chunk_count_words(n)
// words, band after band), added per band to band_cnt[b] and in total to
// *total (all zeroed by the caller); each band's 4096-position counts are
// then replaced by their exclusive prefix.
hipError_t launch_chunk_counts_banded(const JobDev* jobs, int n_jobs, const uint32_t* rects, const uint32_t* order,
                                      int64_t n, int nb, uint32_t* counts, uint32_t* band_cnt, uint32_t* total,
                                      hipStream_t st);

// Key emission in depth order: depth position i's tiles (rows, then columns)
// get consecutive slots, starting after all tiles of the positions before it
// (from the chunk counts of launch_chunk_counts).  With `touched` non-null
// (some frame of the batch uses the ellipse overlap mode) the counts come
// from `touched`, and the tiles of such frames' Gaussians are the box's tiles
// that ellipse_row_span keeps, decided from their records `rec`.
// narrow_keys: tile ids are written as uint16_t (a one-pass tile sort, at
// most 2048 tiles), else as uint32_t.
hipError_t launch_emit(const JobDev* jobs, int n_jobs, int64_t n_flat, const uint32_t* order,
                       const uint32_t* chunk_counts, const uint32_t* depth_rects, const uint32_t* touched,
                       const GaussRec* rec, void* tile_keys, bool narrow_keys, uint32_t* tile_vals,
                       int64_t capacity, uint32_t* counters, hipStream_t st);

// Banded emission: band b's pairs fill the run that starts after the pairs
// of bands 0..b-1 (band_cnt and the chunk counts from
// launch_chunk_counts_banded), with band-local tile ids; positions at or
// beyond `capacity` are dropped and flagged.
hipError_t launch_emit_banded(const JobDev* jobs, int n_jobs, int64_t n_flat, const uint32_t* order,
                              const uint32_t* chunk_counts, const uint32_t* depth_rects, int nb,
                              const uint32_t* band_cnt, uint16_t* tile_keys, uint32_t* tile_vals, int64_t capacity,
                              uint32_t* counters, hipStream_t st);

hipError_t launch_ranges(const uint32_t* sorted_tiles, DevCount n, uint32_t* ranges, int64_t n_tiles,
                         hipStream_t st);

// 64-bit (local tile << 32 | depth key) keys and job-local values of one
// job's sorted pairs [begin, ...), from the job's tiles' ranges.
hipError_t launch_compose_keys(const uint32_t* job_ranges, int64_t tiles, const uint32_t* sorted_vals,
                               const uint32_t* zkey, int64_t begin, int64_t gauss_base, uint64_t* keys_out,
                               uint32_t* vals_out, hipStream_t st);

// Gradient-aware interpolation to scale x scale times the pixels (scale 1..4).
hipError_t launch_gradient_upsample(const float* rgb, const float* dcdx, const float* dcdy, int W, int H, int S,
                                    float* out, hipStream_t st);

// Motion vectors and forward warping: the two cameras in FP64 (source,
// destination) and the raster sizes of both.
struct WarpCams {
    double Rs[9], ts[3], fxs, fys, cxs, cys;
    double Rd[9], td[3], fxd, fyd, cxd, cyd;
    int32_t W, H, Wd, Hd;
};

// Warped outputs on the destination raster; a NULL plane is not written.
struct WarpOut {
    float* rgb;
    float* depth;
    float* dcdx;
    float* dcdy;
    float* weight;
    int32_t* source;
    float* normal;
};

// z-buffer fill, motion vectors + depth-tested splat, resolve.  The workspace
// (16-byte aligned, warp_workspace_bytes) holds the z-buffer and the FP64
// motion vectors.
size_t warp_workspace_bytes(int64_t src_pixels, int64_t dst_pixels);
hipError_t launch_motion_warp(const WarpCams& c, const float* rgb, const float* alpha, const float* depth,
                              const float* dcdx, const float* dcdy, const float* normal, float* motion,
                              const WarpOut& o, void* workspace, hipStream_t st);

// nrm non-null: the normal-blending variant (normal and nv outputs).
hipError_t launch_composite(const JobDev* jobs, int n_jobs, int64_t n_tiles, int64_t n_flat, const GaussRec* rec,
                            const uint32_t* sorted_vals, const uint32_t* ranges, int64_t key_capacity, bool count,
                            const float4* nrm, hipStream_t st);

// Words of the workspace's uint32 counters: the pair count (0), the
// capacity-exceeded flag (1), the compositing work queue's head (2), from
// word 16 the tiles composited per frame of the batch (64 words, one per
// frame of the largest batch) and from word 80 the pairs per tile band
// (kMaxBands words).
constexpr int kQueueHeadWord = 2;
constexpr int kJobDoneWord = 16;
constexpr int kBandCountWord = 80;
constexpr int kCounterWords = kBandCountWord + kMaxBands;

// The same compositing (without the counting and normal outputs) as a
// persistent grid over a work queue of the batch's tiles (counters as above,
// cleared before the pass); frame j's completion is published by a release
// store of seq to done_host[j] (host memory).
hipError_t launch_composite_queue(const JobDev* jobs, int n_jobs, int64_t n_tiles, int64_t n_flat,
                                  const GaussRec* rec, const uint32_t* sorted_vals, const uint32_t* ranges,
                                  int64_t key_capacity, uint32_t* counters, uint32_t* done_host, uint32_t seq,
                                  hipStream_t st);

// Backward: per-Gaussian 2D gradients (du, dv, dA, dB, dC, do, dr, dg, db, dz)
// accumulated into grads2d [n_flat x 10] (zeroed by the caller).
hipError_t launch_composite_bwd(const JobDev* jobs, int n_jobs, int64_t n_tiles, int64_t n_flat, const GaussRec* rec,
                                const uint32_t* sorted_vals, const uint32_t* ranges, const float* dL_drgb,
                                const float* dL_dalpha, const float* dL_ddepth, float* grads2d, hipStream_t st);

// overwrite: write (=) every Gaussian's gradients, zeros where it reaches no
// tile, instead of adding to them.
hipError_t launch_project_bwd(const JobDev* jobs, int n_jobs, int64_t n_flat, const uint32_t* touched,
                              const float* grads2d, float* d_means, float* d_log_scales, float* d_quats,
                              float* d_opac, float* d_sh, bool overwrite, hipStream_t st);

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t st);
// The same fill; its first thread also writes `one` to table[0].
hipError_t launch_fill_u32_job(uint32_t* p, uint32_t value, int64_t n, const JobDev& one, JobDev* table,
                               hipStream_t st);

}  // namespace gs
