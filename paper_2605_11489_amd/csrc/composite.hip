// Front-to-back compositing with the analytic image gradients in the same
// pass (3DGS^3 Sec. 3, Eq. 2-4).
//
// One workgroup per 16x16 tile, one pixel per thread; each of the four
// wavefronts owns an 8x8 quadrant so a splat's footprint lights up as few
// wavefronts as possible.  The tile's depth-sorted list is consumed in
// batches of 256: every thread stages one Gaussian into LDS (FP64 -> tile
// relative float mean, base-2 exponent coefficients) and marks the quadrants
// its alpha >= 1/255 ellipse can reach; each wavefront then walks its own
// list of the batch, two slots per step so that the LDS reads and exponents
// of the pair overlap, reading the records as LDS broadcasts.  A pixel leaves
// its loop when its transmittance would drop below 1e-4; the wavefront leaves
// when all its lanes have, and the workgroup stops staging once every pixel
// is done (barrier count).  Per blended Gaussian the pixel updates C, D
// (Eq. 2), dC (Eq. 3) and dT (Eq. 4); the skip test runs on the exponent, so
// a wavefront whose pixels all miss a splat never issues the exp.
//
// A 960x540 frame has 8160 wavefronts, 8 per SIMD: the kernel is held to 64
// VGPRs so that all of them are resident at once.
//
// The normal-blending variant (k_composite_normals) also stages each
// Gaussian's camera-facing normal in the spare lanes of the z slot and
// accumulates N = sum n alpha T beside the colour; at the end it writes N and
// Nv = -N . r / |r|, r the pixel's ray (the normal maps of Sec. 4.1, 4.2).
//
// Bound: FP32 VALU; nothing here is a dense contraction, so no MFMA.
#include <atomic>

#include "composite_common.hpp"
#include "gs_kernels.hpp"

namespace gs {

constexpr int kCompThreads = 256;
// slot kCompThreads of the staged arrays is a Gaussian no pixel keeps; it
// pads a wavefront's slot list to a whole number of unrolled steps
constexpr int kSlots = kCompThreads + 1;
// slots per step of the walk (the list is read as u16 pairs)
constexpr int kUnroll = 2;

// Per-pixel compositing state (Eq. 2-4): colour, depth, their x/y
// derivatives, transmittance and its derivatives.  The derivatives (dC*,
// dT*) are kept divided by kSlopeToConic, so a blend multiplies the
// exponent's slopes by alpha's weight without the factor; the outputs apply
// it once per pixel.
struct PixelState {
    float T, D, Cr, Cg, Cb, dCxr, dCxg, dCxb, dCyr, dCyg, dCyb, dTx, dTy;
    float Nx, Ny, Nz;   // blended normal (normal-blending variant only)
    float emin;      // alpha exponent a kept Gaussian must reach; +inf once the pixel is done
    uint32_t last;   // list position + 1 of the last blended Gaussian (times 16 unless wide)
    uint32_t n_eval, n_blend;
};

// One kept Gaussian, front to back.  `want` lanes reach alpha >= 1/255; the
// termination test (T would drop below 1e-4) ends a lane without blending.
// Returns true when a lane of the wavefront ended here.
template <bool kCount, bool kNormals>
__device__ __forceinline__ bool blend_slot(PixelState& ps, const char* shb, uint32_t off, uint32_t lastv,
                                           float ex, float ga, float gb, bool want, uint64_t wm) {
    // operands of the blend, read before the exp so their latency overlaps it
    const float4 s2 = *reinterpret_cast<const float4*>(shb + 2 * kSlots * sizeof(float4) + off);
    float z;
    float3 nrm;
    if (kNormals) {
        const float4 s3 = *reinterpret_cast<const float4*>(shb + 3 * kSlots * sizeof(float4) + off);
        z = s3.x;
        nrm = make_float3(s3.y, s3.z, s3.w);
    } else {
        z = *reinterpret_cast<const float*>(shb + 3 * kSlots * sizeof(float4) + off);
    }
    const float ap = fast_exp2(ex);
    const float a = fminf(ap, kAlphaMax);
    const float Tn = __builtin_fmaf(-a, ps.T, ps.T);   // T (1 - alpha), one rounding
    const bool stop = want && Tn < kTMin;
    // (ballot of the compare alone, so the mask needs no materialising)
    const bool any_stop = (__builtin_amdgcn_ballot_w64(Tn < kTMin) & wm) != 0ull;
    // (rare: each pixel stops once; off the blend path, the select costs no
    // instruction per blend)
    if (__builtin_expect(any_stop, 0)) ps.emin = stop ? __builtin_inff() : ps.emin;
    if (want && !stop) {
        const float w = a * ps.T;
        ps.Cr = __builtin_fmaf(s2.y, w, ps.Cr);
        ps.Cg = __builtin_fmaf(s2.z, w, ps.Cg);
        ps.Cb = __builtin_fmaf(s2.w, w, ps.Cb);
        ps.D = __builtin_fmaf(z, w, ps.D);
        if (kNormals) {
            ps.Nx = __builtin_fmaf(nrm.x, w, ps.Nx);
            ps.Ny = __builtin_fmaf(nrm.y, w, ps.Ny);
            ps.Nz = __builtin_fmaf(nrm.z, w, ps.Nz);
        }
        // d alpha/d(x,y) = alpha (A dx + B dy, B dx + C dy), zero at the clamp;
        // the exponent's slopes ga, gb are those terms over kSlopeToConic.
        // dw = alpha dT + T dalpha adds c dw to dC (Eq. 3); Eq. 4,
        // dT' = (1 - alpha) dT - T dalpha, is the same as dT' = dT - dw.
        const float wf = ap < kAlphaMax ? w : 0.f;
        const float wx = __builtin_fmaf(wf, ga, a * ps.dTx);
        const float wy = __builtin_fmaf(wf, gb, a * ps.dTy);
        ps.dCxr = __builtin_fmaf(s2.y, wx, ps.dCxr);
        ps.dCxg = __builtin_fmaf(s2.z, wx, ps.dCxg);
        ps.dCxb = __builtin_fmaf(s2.w, wx, ps.dCxb);
        ps.dCyr = __builtin_fmaf(s2.y, wy, ps.dCyr);
        ps.dCyg = __builtin_fmaf(s2.z, wy, ps.dCyg);
        ps.dCyb = __builtin_fmaf(s2.w, wy, ps.dCyb);
        ps.dTx -= wx;
        ps.dTy -= wy;
        ps.T = Tn;
        if (kCount) ++ps.n_blend;
        ps.last = lastv;
    }
    return any_stop;
}

// The compositing workgroup's LDS, shared by the kernels of this file.  The
// staged batch is laid out so that one byte offset off = 16 k addresses slot
// k of every array: (mu, mv, a, b) at off, (c, lo, A, B) at 16 kSlots +
// off, (C, r, g, b) at 32 kSlots + off, z at 48 kSlots + off.
__shared__ float4 lds_stage[4][kSlots];
__shared__ uint8_t lds_mask[kCompThreads];
__shared__ uint16_t lds_list[4][kCompThreads + kUnroll];

// The padding slot (zero conic, log2 opacity -inf, so its exponent is -inf),
// once per workgroup before its first tile: staging never reaches it.  Every
// lane of wavefront 0 stores the same values (a branch that is uniform
// within each wavefront).
__device__ __forceinline__ void write_padding_slot() {
    if (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0) {
        lds_stage[0][kCompThreads] = make_float4(0.f, 0.f, 0.f, 0.f);
        lds_stage[1][kCompThreads] = make_float4(0.f, -__builtin_inff(), 0.f, 0.f);
    }
}

// One 16x16 tile (global tile id gt), after write_padding_slot.
// kWide: tile lists may reach 2^28 entries, so the last blended position is
// kept as a plain index instead of 16 times the index.
template <bool kCount, bool kWide, bool kNormals>
__device__ __forceinline__ void composite_tile(const JobDev* __restrict__ jobs, int n_jobs,
                                               const GaussRec* __restrict__ rec,
                                               const uint32_t* __restrict__ sorted_vals,
                                               const uint32_t* __restrict__ ranges, int64_t n_flat,
                                               const float4* __restrict__ nrm, const int gt) {
    float4 (&sh)[4][kSlots] = lds_stage;
    uint8_t (&smask)[kCompThreads] = lds_mask;
    uint16_t (&slist)[4][kCompThreads + kUnroll] = lds_list;

    const int j = find_job_tile(jobs, n_jobs, gt);
    const JobDev& jb = jobs[j];
    const int lt = gt - jb.tile_base;
    const int tx = lt % jb.tiles_x;
    const int ty = lt / jb.tiles_x;
    const int W = jb.width, H = jb.height;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int lx = ((wave & 1) << 3) + (lane & 7);
    const int ly = ((wave >> 1) << 3) + (lane >> 3);
    const int ix = tx * kTile + lx, iy = ty * kTile + ly;
    const bool inside = ix < W && iy < H;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const double x0 = (double)(tx * kTile), y0 = (double)(ty * kTile);

    const uint32_t s = ranges[2 * gt], e = ranges[2 * gt + 1];

    PixelState ps;
    ps.T = 1.f;
    ps.D = ps.Cr = ps.Cg = ps.Cb = 0.f;
    ps.dCxr = ps.dCxg = ps.dCxb = ps.dCyr = ps.dCyg = ps.dCyb = 0.f;
    ps.dTx = ps.dTy = 0.f;
    ps.Nx = ps.Ny = ps.Nz = 0.f;
    ps.last = 0;
    ps.n_eval = ps.n_blend = 0;
    // A pixel keeps a Gaussian when its alpha exponent reaches emin; a
    // finished (or off-image) pixel has emin = +inf, so "keep" is one compare.
    ps.emin = inside ? kLog2AlphaMin : __builtin_inff();
    bool wave_done = __builtin_amdgcn_ballot_w64(inside) == 0ull;
    const char* shb = reinterpret_cast<const char*>(&sh[0][0]);

    for (uint32_t b0 = s; b0 < e; b0 += kCompThreads) {
        if (__syncthreads_count(ps.emin == __builtin_inff()) == kCompThreads) break;
        // staging and list building run at raised wave priority: the
        // workgroup's four wavefronts wait for them at the barriers, while the
        // other workgroups' walks on the CU can wait (-0.6 us at 960x540)
        __builtin_amdgcn_s_setprio(3);
        const uint32_t idx = b0 + tid;
        uint32_t qm = 0;
        if (idx < e) {
            uint32_t g = sorted_vals[idx];
            g = (int64_t)g < n_flat ? g : 0u;
            const GaussRec r = rec[g];
            Staged st = stage_gaussian(r, x0, y0);
            if (kNormals) {
                const float4 n = nrm[g];
                st.s3.y = n.x;
                st.s3.z = n.y;
                st.s3.w = n.z;
            }
            sh[0][tid] = st.s0;
            sh[1][tid] = st.s1;
            sh[2][tid] = st.s2;
            sh[3][tid] = st.s3;
            // the counting variant keeps every pair so it counts evaluations exactly
            qm = kCount ? 0xFu : quadrant_mask(r, st.s0.x, st.s0.y, st.s1.y);
        }
        smask[tid] = (uint8_t)qm;
        __syncthreads();
        // each wavefront lists, in order, the batch slots that can reach its quadrant
        int nb = 0;
#pragma unroll
        for (int c = 0; c < kCompThreads / 64; ++c) {
            const bool bit = (smask[c * 64 + lane] >> wave) & 1u;
            const uint64_t bm = __builtin_amdgcn_ballot_w64(bit);
            const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
            if (bit) slist[wave][nb + __popcll(bm & lt)] = (uint16_t)((c * 64 + lane) * (int)sizeof(float4));
            nb += __popcll(bm);
        }
        if (lane < kUnroll) slist[wave][nb + lane] = (uint16_t)(kCompThreads * sizeof(float4));
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
        // position + 1 in the tile list of slot 0, times 16 unless kWide
        const uint32_t base1 = kWide ? b0 - s + 1u : (b0 - s + 1u) * (uint32_t)sizeof(float4);
        // Every lane walks the batch in lock step, kUnroll slots per step so
        // the LDS reads and exponents of the step overlap.  A Gaussian that no
        // live lane of the wavefront keeps (alpha >= 1/255) costs no branch
        // into the blend; otherwise its keeping lanes blend it under the
        // execution mask.
        for (int i = 0; i < nb && !wave_done; i += kUnroll) {
            uint32_t off[kUnroll];
            {
                const uint32_t pr = *reinterpret_cast<const uint32_t*>(&slist[wave][i]);
                off[0] = pr & 0xFFFFu;
                off[1] = pr >> 16;
            }
            float ex[kUnroll], ga[kUnroll], gb[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const float4 s0 = *reinterpret_cast<const float4*>(shb + off[u]);
                const float2 s1 = *reinterpret_cast<const float2*>(shb + kSlots * sizeof(float4) + off[u]);
                ex[u] = alpha_exponent_slopes(s0, s1, s0.x - px, s0.y - py, ga[u], gb[u]);
            }
            bool stopped = false;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (kCount && ps.emin != __builtin_inff() && (u == 0 || i + u < nb)) ++ps.n_eval;
                const bool want = ex[u] >= ps.emin;
                const uint64_t wm = __builtin_amdgcn_ballot_w64(want);
                if (wm != 0ull) {
                    const uint32_t lastv = kWide ? base1 + (off[u] >> 4) : base1 + off[u];
                    stopped |= blend_slot<kCount, kNormals>(ps, shb, off[u], lastv, ex[u], ga[u], gb[u], want, wm);
                }
            }
            if (stopped) wave_done = __builtin_amdgcn_ballot_w64(ps.emin != __builtin_inff()) == 0ull;
        }
    }

    float T = ps.T, D = ps.D, Cr = ps.Cr, Cg = ps.Cg, Cb = ps.Cb;
    float dCxr = ps.dCxr, dCxg = ps.dCxg, dCxb = ps.dCxb, dCyr = ps.dCyr, dCyg = ps.dCyg, dCyb = ps.dCyb;
    float dTx = ps.dTx, dTy = ps.dTy;
    const uint32_t last = ps.last, n_eval = ps.n_eval, n_blend = ps.n_blend;
    if (!inside) return;
    const int64_t HW = (int64_t)W * H;
    const int64_t p = (int64_t)iy * W + ix;
    const float bgr = jb.bg[0], bgg = jb.bg[1], bgb = jb.bg[2];
    if (jb.rgb) {
        jb.rgb[p] = __builtin_fmaf(T, bgr, Cr);
        jb.rgb[HW + p] = __builtin_fmaf(T, bgg, Cg);
        jb.rgb[2 * HW + p] = __builtin_fmaf(T, bgb, Cb);
    }
    if (jb.alpha) jb.alpha[p] = 1.f - T;
    if (jb.depth) jb.depth[p] = D;
    if (jb.dcdx) {
        jb.dcdx[p] = kSlopeToConic * __builtin_fmaf(dTx, bgr, dCxr);
        jb.dcdx[HW + p] = kSlopeToConic * __builtin_fmaf(dTx, bgg, dCxg);
        jb.dcdx[2 * HW + p] = kSlopeToConic * __builtin_fmaf(dTx, bgb, dCxb);
    }
    if (jb.dcdy) {
        jb.dcdy[p] = kSlopeToConic * __builtin_fmaf(dTy, bgr, dCyr);
        jb.dcdy[HW + p] = kSlopeToConic * __builtin_fmaf(dTy, bgg, dCyg);
        jb.dcdy[2 * HW + p] = kSlopeToConic * __builtin_fmaf(dTy, bgb, dCyb);
    }
    jb.final_T[p] = T;
    jb.n_contrib[p] = kWide ? last : last >> 4;
    if (kCount) {
        if (jb.n_evaluated) jb.n_evaluated[p] = n_eval;
        if (jb.n_blended) jb.n_blended[p] = n_blend;
    }
    if (kNormals) {
        const float Nx = ps.Nx, Ny = ps.Ny, Nz = ps.Nz;
        if (jb.normal) {
            jb.normal[p] = Nx;
            jb.normal[HW + p] = Ny;
            jb.normal[2 * HW + p] = Nz;
        }
        if (jb.nv) {
            // once per pixel: the ray in FP64
            const double rx = ((double)ix + 0.5 - jb.cx) / jb.fx;
            const double ry = ((double)iy + 0.5 - jb.cy) / jb.fy;
            const double inv = 1.0 / sqrt(rx * rx + ry * ry + 1.0);
            jb.nv[p] = (float)(-((double)Nx * rx + (double)Ny * ry + (double)Nz) * inv);
        }
    }
}

template <bool kCount, bool kWide>
__global__ void __launch_bounds__(kCompThreads) __attribute__((amdgpu_waves_per_eu(8)))
k_composite(const JobDev* __restrict__ jobs, int n_jobs, const GaussRec* __restrict__ rec,
            const uint32_t* __restrict__ sorted_vals, const uint32_t* __restrict__ ranges, int64_t n_flat) {
    write_padding_slot();
    composite_tile<kCount, kWide, false>(jobs, n_jobs, rec, sorted_vals, ranges, n_flat, nullptr, blockIdx.x);
}

template <bool kCount, bool kWide>
__global__ void __launch_bounds__(kCompThreads)
k_composite_normals(const JobDev* __restrict__ jobs, int n_jobs, const GaussRec* __restrict__ rec,
                    const uint32_t* __restrict__ sorted_vals, const uint32_t* __restrict__ ranges, int64_t n_flat,
                    const float4* __restrict__ nrm) {
    write_padding_slot();
    composite_tile<kCount, kWide, true>(jobs, n_jobs, rec, sorted_vals, ranges, n_flat, nrm, blockIdx.x);
}

// Persistent compositing over a device work queue, for the serving loop:
// a grid of at most as many workgroups as the device holds at once pulls
// the tiles of every frame of a batch from one counter in the workspace
// (counters[kQueueHeadWord]) after the first round of one tile per
// workgroup, frame after frame in batch order, so the batch's first frames
// finish first.  Each frame but the batch's last is
// published as soon as it is complete: a workgroup that leaves a frame (its
// next tile belongs to a later frame, or the queue is empty) adds the tiles
// it composited of it to the frame's count (counters[kJobDoneWord + j]), and
// the one that completes the count stores seq into done_host[j], host memory
// that the server polls.  Before that, every wavefront waits until its
// stores have reached the L2 the workgroup shares, and thread 0 releases at
// device scope (a writeback of that L2) before the count and at system scope
// before the flag, so a reader that sees the flag and then reads the frame
// (from any later launch or copy) sees all of it.  The writeback is what a
// publication costs (a workgroup's per frame, not per tile), so the batch's
// last frame, which is complete when the batch is, is never published.
// Nothing waits on another workgroup: a workgroup leaves once the counter
// has passed the last tile.  A batch whose pairs overflowed the key capacity
// (counters[1], set by the emission) composites nothing and publishes
// nothing: its frames are re-run.
// One add for the whole wavefront (lane 0 adds n, the others 0); every lane
// returns the counter's previous value.
__device__ __forceinline__ uint32_t wave_fetch_add(uint32_t* p, uint32_t n, int memorder) {
    const uint32_t v = __lane_id() == 0 ? n : 0u;
    const uint32_t old = memorder == __ATOMIC_ACQ_REL
                             ? __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT)
                             : __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_amdgcn_readfirstlane(old);
}

template <bool kWide>
__global__ void __launch_bounds__(kCompThreads) __attribute__((amdgpu_waves_per_eu(8)))
k_composite_queue(const JobDev* __restrict__ jobs, int n_jobs, const GaussRec* __restrict__ rec,
                  const uint32_t* __restrict__ sorted_vals, const uint32_t* __restrict__ ranges, int64_t n_flat,
                  uint32_t n_tiles, uint32_t* counters, uint32_t* done_host, uint32_t seq) {
    __shared__ uint32_t s_item;
    if (counters[1] != 0u) return;
    // Wavefront 0 claims tiles and publishes frames with every lane active
    // (a branch uniform within each wavefront), so no barrier is ever
    // reached by part of a wavefront.
    const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0;
    // A workgroup's first tile is its own index (the grid's workgroups all
    // start at once, and claiming those through one counter would serialise
    // them on it); the tiles after the grid's first round are claimed from
    // the counter as workgroups free up.
    const uint32_t grid = gridDim.x;
    uint32_t gt = blockIdx.x;
    write_padding_slot();
    uint32_t pending = 0;   // tiles of the current frame composited and not yet published
    // a workgroup claims at most n_tiles tiles, which bounds the loop as well
    for (uint32_t claimed = 0; gt < n_tiles && claimed < n_tiles; ++claimed) {
        composite_tile<false, kWide, false>(jobs, n_jobs, rec, sorted_vals, ranges, n_flat, nullptr, (int)gt);
        ++pending;
        uint32_t nx = n_tiles;
        if (grid < n_tiles) {
            __syncthreads();
            if (wave0) s_item = grid + wave_fetch_add(&counters[kQueueHeadWord], 1u, __ATOMIC_RELAXED);
            __syncthreads();
            nx = __builtin_amdgcn_readfirstlane(s_item);
        }
        const int j = find_job_tile(jobs, n_jobs, gt);
        if (nx >= n_tiles || find_job_tile(jobs, n_jobs, nx) != j) {
            if (j + 1 < n_jobs) {
                __builtin_amdgcn_s_waitcnt(0);   // this wavefront's stores are in the L2
                __syncthreads();
                if (wave0) {
                    const uint32_t nt = (uint32_t)(jobs[j].tiles_x * jobs[j].tiles_y);
                    const uint32_t done = wave_fetch_add(&counters[kJobDoneWord + j], pending, __ATOMIC_ACQ_REL);
                    if (done + pending == nt)
                        __hip_atomic_store(&done_host[j], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                __syncthreads();
            }
            pending = 0;
        }
        gt = nx;
    }
}

hipError_t launch_composite_queue(const JobDev* jobs, int n_jobs, int64_t n_tiles, int64_t n_flat,
                                  const GaussRec* rec, const uint32_t* sorted_vals, const uint32_t* ranges,
                                  int64_t key_capacity, uint32_t* counters, uint32_t* done_host, uint32_t seq,
                                  hipStream_t st) {
    if (n_tiles == 0) return hipSuccess;
    // resident workgroups per device, once per device (a host query per
    // batch would cost more than a small frame's compositing)
    constexpr int kMaxDevices = 64;
    static std::atomic<int64_t> resident_cache[kMaxDevices];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int64_t resident = dev < kMaxDevices ? resident_cache[dev].load(std::memory_order_relaxed) : 0;
    if (resident <= 0) {
        int cus = 0, per_cu = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        // (both instantiations have the same resources)
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_composite_queue<false>,
                                                             kCompThreads, 0);
        if (e != hipSuccess) return e;
        resident = (int64_t)(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
        if (dev < kMaxDevices) resident_cache[dev].store(resident, std::memory_order_relaxed);
    }
    const bool wide = key_capacity >= ((int64_t)1 << 28);
    const dim3 grid((unsigned)(n_tiles < resident ? n_tiles : resident)), block(kCompThreads);
    const uint32_t nt = (uint32_t)n_tiles;
    if (wide)
        hipLaunchKernelGGL((k_composite_queue<true>), grid, block, 0, st, jobs, n_jobs, rec, sorted_vals, ranges,
                           n_flat, nt, counters, done_host, seq);
    else
        hipLaunchKernelGGL((k_composite_queue<false>), grid, block, 0, st, jobs, n_jobs, rec, sorted_vals, ranges,
                           n_flat, nt, counters, done_host, seq);
    return hipGetLastError();
}

hipError_t launch_composite(const JobDev* jobs, int n_jobs, int64_t n_tiles, int64_t n_flat, const GaussRec* rec,
                            const uint32_t* sorted_vals, const uint32_t* ranges, int64_t key_capacity, bool count,
                            const float4* nrm, hipStream_t st) {
    if (n_tiles == 0) return hipSuccess;
    const bool wide = key_capacity >= ((int64_t)1 << 28);
    const dim3 grid((unsigned)n_tiles), block(kCompThreads);
    if (nrm) {
        if (count && wide)
            hipLaunchKernelGGL((k_composite_normals<true, true>), grid, block, 0, st, jobs, n_jobs, rec, sorted_vals,
                               ranges, n_flat, nrm);
        else if (count)
            hipLaunchKernelGGL((k_composite_normals<true, false>), grid, block, 0, st, jobs, n_jobs, rec, sorted_vals,
                               ranges, n_flat, nrm);
        else if (wide)
            hipLaunchKernelGGL((k_composite_normals<false, true>), grid, block, 0, st, jobs, n_jobs, rec, sorted_vals,
                               ranges, n_flat, nrm);
        else
            hipLaunchKernelGGL((k_composite_normals<false, false>), grid, block, 0, st, jobs, n_jobs, rec,
                               sorted_vals, ranges, n_flat, nrm);
        return hipGetLastError();
    }
    if (count && wide)
        hipLaunchKernelGGL((k_composite<true, true>), grid, block, 0, st, jobs, n_jobs, rec, sorted_vals, ranges, n_flat);
    else if (count)
        hipLaunchKernelGGL((k_composite<true, false>), grid, block, 0, st, jobs, n_jobs, rec, sorted_vals, ranges, n_flat);
    else if (wide)
        hipLaunchKernelGGL((k_composite<false, true>), grid, block, 0, st, jobs, n_jobs, rec, sorted_vals, ranges, n_flat);
    else
        hipLaunchKernelGGL((k_composite<false, false>), grid, block, 0, st, jobs, n_jobs, rec, sorted_vals, ranges, n_flat);
    return hipGetLastError();
}

}  // namespace gs
