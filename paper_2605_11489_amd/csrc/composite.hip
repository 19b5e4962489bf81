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
// derivatives, transmittance and its derivatives.
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
                                           float ex, float dx, float dy, bool want, uint64_t wm) {
    // operands of the blend, read before the exp so their latency overlaps it
    const float2 gab = *reinterpret_cast<const float2*>(shb + kSlots * sizeof(float4) + 8 + off);
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
    if (any_stop) ps.emin = stop ? __builtin_inff() : ps.emin;
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
        // d alpha/d(x,y) = alpha (A dx + B dy, B dx + C dy), zero at the clamp.
        // dw = alpha dT + T dalpha adds c dw to dC (Eq. 3); Eq. 4,
        // dT' = (1 - alpha) dT - T dalpha, is the same as dT' = dT - dw.
        const float wf = ap < kAlphaMax ? w : 0.f;
        const float ga = __builtin_fmaf(gab.x, dx, gab.y * dy);
        const float gb = __builtin_fmaf(gab.y, dx, s2.x * dy);
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

// kWide: tile lists may reach 2^28 entries, so the last blended position is
// kept as a plain index instead of 16 times the index.
template <bool kCount, bool kWide, bool kNormals>
__device__ __forceinline__ void composite_tile(const JobDev* __restrict__ jobs, int n_jobs,
                                               const GaussRec* __restrict__ rec,
                                               const uint32_t* __restrict__ sorted_vals,
                                               const uint32_t* __restrict__ ranges, int64_t n_flat,
                                               const float4* __restrict__ nrm) {
    // staged batch, laid out so that one byte offset off = 16 k addresses
    // slot k of every array: (mu, mv, a2, b2) at off, (c2, lo, A, B) at
    // 16 kSlots + off, (C, r, g, b) at 32 kSlots + off, z at 48 kSlots + off
    __shared__ float4 sh[4][kSlots];
    __shared__ uint8_t smask[kCompThreads];
    __shared__ uint16_t slist[4][kCompThreads + kUnroll];

    const int gt = blockIdx.x;
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
    if (tid == 0) {
        // the padding slot: zero conic, log2 opacity -inf, so its exponent is -inf
        sh[0][kCompThreads] = make_float4(0.f, 0.f, 0.f, 0.f);
        sh[1][kCompThreads] = make_float4(0.f, -__builtin_inff(), 0.f, 0.f);
    }
    const char* shb = reinterpret_cast<const char*>(&sh[0][0]);

    for (uint32_t b0 = s; b0 < e; b0 += kCompThreads) {
        if (__syncthreads_count(ps.emin == __builtin_inff()) == kCompThreads) break;
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
            float ex[kUnroll], dx[kUnroll], dy[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const float4 s0 = *reinterpret_cast<const float4*>(shb + off[u]);
                const float2 s1 = *reinterpret_cast<const float2*>(shb + kSlots * sizeof(float4) + off[u]);
                dx[u] = s0.x - px;
                dy[u] = s0.y - py;
                const float m = s0.w * dy[u];
                const float n = __builtin_fmaf(s0.z, dx[u], m);
                const float k = s1.x * dy[u];
                const float l = __builtin_fmaf(k, dy[u], s1.y);
                ex[u] = __builtin_fmaf(dx[u], n, l);
            }
            bool stopped = false;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (kCount && ps.emin != __builtin_inff() && (u == 0 || i + u < nb)) ++ps.n_eval;
                const bool want = ex[u] >= ps.emin;
                const uint64_t wm = __builtin_amdgcn_ballot_w64(want);
                if (wm != 0ull) {
                    const uint32_t lastv = kWide ? base1 + (off[u] >> 4) : base1 + off[u];
                    stopped |= blend_slot<kCount, kNormals>(ps, shb, off[u], lastv, ex[u], dx[u], dy[u], want, wm);
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
        jb.dcdx[p] = __builtin_fmaf(dTx, bgr, dCxr);
        jb.dcdx[HW + p] = __builtin_fmaf(dTx, bgg, dCxg);
        jb.dcdx[2 * HW + p] = __builtin_fmaf(dTx, bgb, dCxb);
    }
    if (jb.dcdy) {
        jb.dcdy[p] = __builtin_fmaf(dTy, bgr, dCyr);
        jb.dcdy[HW + p] = __builtin_fmaf(dTy, bgg, dCyg);
        jb.dcdy[2 * HW + p] = __builtin_fmaf(dTy, bgb, dCyb);
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
    composite_tile<kCount, kWide, false>(jobs, n_jobs, rec, sorted_vals, ranges, n_flat, nullptr);
}

template <bool kCount, bool kWide>
__global__ void __launch_bounds__(kCompThreads)
k_composite_normals(const JobDev* __restrict__ jobs, int n_jobs, const GaussRec* __restrict__ rec,
                    const uint32_t* __restrict__ sorted_vals, const uint32_t* __restrict__ ranges, int64_t n_flat,
                    const float4* __restrict__ nrm) {
    composite_tile<kCount, kWide, true>(jobs, n_jobs, rec, sorted_vals, ranges, n_flat, nrm);
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
