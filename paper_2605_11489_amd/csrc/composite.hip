// Front-to-back compositing with the analytic image gradients in the same
// pass (3DGS^3 Sec. 3, Eq. 2-4).
//
// One workgroup per 16x16 tile, one pixel per thread; each of the four
// wavefronts owns an 8x8 quadrant so a splat's footprint lights up as few
// wavefronts as possible.  The tile's depth-sorted list is consumed in
// batches of 256: every thread stages one Gaussian into LDS (FP64 -> tile
// relative float mean, base-2 exponent coefficients), then every pixel walks
// the batch reading the records as LDS broadcasts.  A pixel leaves its loop
// when its transmittance would drop below 1e-4; the wavefront leaves when all
// its lanes have, and the workgroup stops staging once every pixel is done
// (barrier count).  Per blended Gaussian the pixel updates C, D (Eq. 2),
// dC (Eq. 3) and dT (Eq. 4); the skip test runs on the exponent, so a
// wavefront whose pixels all miss a splat never issues the exp.
//
// Bound: FP32 VALU; nothing here is a dense contraction, so no MFMA.
#include "composite_common.hpp"
#include "gs_kernels.hpp"

namespace gs {

constexpr int kCompThreads = 256;

template <bool kCount>
__global__ void __launch_bounds__(kCompThreads) k_composite(const JobDev* __restrict__ jobs, int n_jobs,
                                                            const GaussRec* __restrict__ rec,
                                                            const uint32_t* __restrict__ sorted_vals,
                                                            const uint32_t* __restrict__ ranges,
                                                            int64_t n_flat) {
    __shared__ float4 sh0[kCompThreads];
    __shared__ float4 sh1[kCompThreads];
    __shared__ float4 sh2[kCompThreads];
    __shared__ float sh3[kCompThreads];
    __shared__ uint8_t smask[kCompThreads];
    __shared__ uint8_t slist[4][kCompThreads];

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

    float T = 1.f, D = 0.f;
    float Cr = 0.f, Cg = 0.f, Cb = 0.f;
    float dCxr = 0.f, dCxg = 0.f, dCxb = 0.f, dCyr = 0.f, dCyg = 0.f, dCyb = 0.f;
    float dTx = 0.f, dTy = 0.f;
    uint32_t last = 0;
    uint32_t n_eval = 0, n_blend = 0;
    // A pixel keeps a Gaussian when its alpha exponent reaches emin; a
    // finished (or off-image) pixel has emin = +inf, so "keep" is one compare.
    float emin = inside ? kLog2AlphaMin : __builtin_inff();
    bool wave_done = !inside && __builtin_amdgcn_ballot_w64(inside) == 0ull;

    for (uint32_t b0 = s; b0 < e; b0 += kCompThreads) {
        if (__syncthreads_count(emin == __builtin_inff()) == kCompThreads) break;
        const uint32_t idx = b0 + tid;
        uint32_t qm = 0;
        if (idx < e) {
            uint32_t g = sorted_vals[idx];
            g = (int64_t)g < n_flat ? g : 0u;
            const GaussRec r = rec[g];
            const Staged st = stage_gaussian(r, x0, y0);
            sh0[tid] = st.s0;
            sh1[tid] = st.s1;
            sh2[tid] = st.s2;
            sh3[tid] = st.s3.x;
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
            if (bit) slist[wave][nb + __popcll(bm & lt)] = (uint8_t)(c * 64 + lane);
            nb += __popcll(bm);
        }
        __syncthreads();
        // Every lane walks the batch in lock step.  A Gaussian that no live
        // lane of the wavefront keeps (alpha >= 1/255) is skipped with one
        // scalar branch; otherwise the blend runs predicated, with alpha = 0
        // (an exact no-op on every accumulator) on the lanes that skip it.
        for (int i = 0; i < nb && !wave_done; ++i) {
            const int k = slist[wave][i];
            const float4 s0 = sh0[k];
            const float4 s1 = sh1[k];
            const float dx = s0.x - px;
            const float dy = s0.y - py;
            const float ex = alpha_exponent(s0, s1, dx, dy);
            if (kCount && emin != __builtin_inff()) ++n_eval;
            const bool want = ex >= emin;
            if (__builtin_amdgcn_ballot_w64(want) == 0ull) continue;
            const float ap = fast_exp2(ex);
            float a = want ? fminf(ap, kAlphaMax) : 0.f;
            float Tn = T * (1.f - a);
            const bool stop = want && Tn < kTMin;
            if (__builtin_amdgcn_ballot_w64(stop) != 0ull) {
                // the stopping Gaussian is not blended and the pixel ends
                a = stop ? 0.f : a;
                Tn = stop ? T : Tn;
                emin = stop ? __builtin_inff() : emin;
                wave_done = __builtin_amdgcn_ballot_w64(emin != __builtin_inff()) == 0ull;
            }
            const float4 s2 = sh2[k];
            const float z = sh3[k];
            const float w = a * T;
            Cr = __builtin_fmaf(s2.y, w, Cr);
            Cg = __builtin_fmaf(s2.z, w, Cg);
            Cb = __builtin_fmaf(s2.w, w, Cb);
            D = __builtin_fmaf(z, w, D);
            // d alpha/d(x,y) = alpha (A dx + B dy, B dx + C dy), zero at the clamp.
            // dw = dT alpha + T dalpha = alpha (dT + T g) adds c dw to dC (Eq. 3);
            // Eq. 4, dT' = (1 - alpha) dT - T dalpha, is the same as dT' = dT - dw.
            const bool free = ap < kAlphaMax;
            const float ga = free ? __builtin_fmaf(s1.z, dx, s1.w * dy) : 0.f;
            const float gb = free ? __builtin_fmaf(s1.w, dx, s2.x * dy) : 0.f;
            const float wx = a * __builtin_fmaf(T, ga, dTx);
            const float wy = a * __builtin_fmaf(T, gb, dTy);
            dCxr = __builtin_fmaf(s2.y, wx, dCxr);
            dCxg = __builtin_fmaf(s2.z, wx, dCxg);
            dCxb = __builtin_fmaf(s2.w, wx, dCxb);
            dCyr = __builtin_fmaf(s2.y, wy, dCyr);
            dCyg = __builtin_fmaf(s2.z, wy, dCyg);
            dCyb = __builtin_fmaf(s2.w, wy, dCyb);
            dTx -= wx;
            dTy -= wy;
            T = Tn;
            if (kCount && a > 0.f) ++n_blend;
            last = a > 0.f ? b0 - s + (uint32_t)k + 1u : last;
        }
    }

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
    jb.n_contrib[p] = last;
    if (kCount) {
        if (jb.n_evaluated) jb.n_evaluated[p] = n_eval;
        if (jb.n_blended) jb.n_blended[p] = n_blend;
    }
}

hipError_t launch_composite(const JobDev* jobs, int n_jobs, int64_t n_tiles, int64_t n_flat, const GaussRec* rec,
                            const uint32_t* sorted_vals, const uint32_t* ranges, bool count, hipStream_t st) {
    if (n_tiles == 0) return hipSuccess;
    if (count)
        hipLaunchKernelGGL(k_composite<true>, dim3((unsigned)n_tiles), dim3(kCompThreads), 0, st, jobs, n_jobs, rec,
                           sorted_vals, ranges, n_flat);
    else
        hipLaunchKernelGGL(k_composite<false>, dim3((unsigned)n_tiles), dim3(kCompThreads), 0, st, jobs, n_jobs,
                           rec, sorted_vals, ranges, n_flat);
    return hipGetLastError();
}

}  // namespace gs
