// Backward (adjoint) pass of the rasterizer with respect to the Gaussian
// parameters, for a loss on the rendered rgb, alpha and depth (3DGS^3 Sec. 3,
// Eq. 1-2; the adjoint is this library's own, the paper trains networks on
// the rendered images but gives no rasterizer backward).
//
// k_composite_bwd: one workgroup per 16x16 tile, the forward's pixel layout.
// Each pixel walks its list backwards from its last blended Gaussian
// (n_contrib), recomputing alpha with the forward's own staging, quadrant
// culling and arithmetic (so every skip decision repeats bit for bit) and
// recovering the transmittance in front of each Gaussian,
// T_i = T_{i+1} / (1 - alpha_i) (reciprocal with one Newton step), instead
// of storing it.  Per Gaussian the
// 10 per-pixel partials (d/du, d/dv, d/dA, d/dB, d/dC, d/do, d/dr, d/dg,
// d/db, d/dz) are summed over each wavefront by halving (lane swaps, then
// DPP adds within rows), over the tile's four wavefronts with LDS float
// atomics (one accumulator per batch of 64 staged Gaussians: 6.5 KB of LDS
// per workgroup, so eight wavefronts per SIMD stay resident), and added to
// the Gaussian's global accumulator with one float atomic per component and
// tile.
//
// k_project_bwd: one thread per Gaussian, the adjoint of the projection in
// FP64 (conic inverse, EWA product, Jacobian, view transform, Sigma = M M^T,
// M = R(q) diag(exp(s))) and FP32 for the sigmoid and the SH colour with its
// view-direction dependence.
#include "composite_common.hpp"
#include "gs_kernels.hpp"

namespace gs {

namespace {

constexpr int kBwdThreads = 256;
constexpr int kG2 = 10;   // per-Gaussian 2D gradient components
// row stride of the per-batch LDS accumulator: odd, so the four rows' sums
// of one Gaussian (different components) fall in different banks
#ifndef GS_BWD_BATCH
#define GS_BWD_BATCH 64
#endif
constexpr int kBwdBatch = GS_BWD_BATCH;   // Gaussians staged per batch (a multiple of 64, at most kBwdThreads)
constexpr int kAccStride = kBwdBatch + 1;

// v + the value DPP control CTRL brings from another lane (full row and bank
// masks, so the move folds into one v_add_f32_dpp)
template <int CTRL>
__device__ __forceinline__ float add_dpp(float v) {
    const int t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false);
    return v + __int_as_float(t);
}

// a and b after a cross-lane swap, added: v_permlane32_swap exchanges the
// upper 32 lanes of a with the lower 32 lanes of b, so the sum holds a's
// two halves added in lanes 0-31 and b's in lanes 32-63; v_permlane16_swap
// does the same for the odd rows of a and the even rows of b, giving rows
// (a0 + a1, b0 + b1, a2 + a3, b2 + b3).
__device__ __forceinline__ float swap32_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum of each of the 10 values over the 64 lanes of a full wavefront, by
// halving: five swap-adds across the halves leave value k in lanes 0-31 and
// value k + 5 in lanes 32-63 of register k; three swap-adds across row
// pairs leave four values per register, one per 16-lane row (rows of q[0]:
// 0, 1, 5, 6; of q[1]: 2, 3, 7, 8; of q[2]: 4, 4, 9, 9); four DPP adds per
// register then give every lane its row's total.  22 cross-lane operations
// and as many adds, where a separate 64-lane reduction per value takes 60 of
// each.
__device__ __forceinline__ void wave_sums_by_row(const float* v, float* q) {
    const float h0 = swap32_add(v[0], v[5]);
    const float h1 = swap32_add(v[1], v[6]);
    const float h2 = swap32_add(v[2], v[7]);
    const float h3 = swap32_add(v[3], v[8]);
    const float h4 = swap32_add(v[4], v[9]);
    q[0] = swap16_add(h0, h1);
    q[1] = swap16_add(h2, h3);
    q[2] = swap16_add(h4, h4);
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = add_dpp<0xB1>(q[r]);    // quad_perm [1, 0, 3, 2]
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = add_dpp<0x4E>(q[r]);    // quad_perm [2, 3, 0, 1]
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = add_dpp<0x141>(q[r]);   // row_half_mirror
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = add_dpp<0x140>(q[r]);   // row_mirror
}

}  // namespace

__global__ void __launch_bounds__(kBwdThreads) k_composite_bwd(const JobDev* __restrict__ jobs, int n_jobs,
                                                               const GaussRec* __restrict__ rec,
                                                               const uint32_t* __restrict__ sorted_vals,
                                                               const uint32_t* __restrict__ ranges, int64_t n_flat,
                                                               const float* __restrict__ dL_drgb,
                                                               const float* __restrict__ dL_dalpha,
                                                               const float* __restrict__ dL_ddepth,
                                                               float* __restrict__ grads2d) {
    __shared__ float4 sh0[kBwdBatch];
    __shared__ float4 sh1[kBwdBatch];
    __shared__ float4 sh2[kBwdBatch];
    __shared__ float2 sh3[kBwdBatch];
    __shared__ uint32_t shg[kBwdBatch];
    __shared__ float wacc[kG2][kAccStride];
    __shared__ uint64_t qbits[kBwdBatch / 64][4];
    __shared__ uint32_t smax;

    const int gt = blockIdx.x;
    const int j = find_job_tile(jobs, n_jobs, gt);
    const JobDev& jb = jobs[j];
    const int lt = gt - jb.tile_base;
    const int tx = lt % jb.tiles_x, ty = lt / jb.tiles_x;
    const int W = jb.width, H = jb.height;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int lx = ((wave & 1) << 3) + (lane & 7);
    const int ly = ((wave >> 1) << 3) + (lane >> 3);
    const int ix = tx * kTile + lx, iy = ty * kTile + ly;
    const bool inside = ix < W && iy < H;
    const float px = (float)lx + 0.5f, py = (float)ly + 0.5f;
    const double x0 = (double)(tx * kTile), y0 = (double)(ty * kTile);
    const uint32_t s = ranges[2 * gt];

    const int64_t HW = (int64_t)W * H;
    const int64_t p = (int64_t)iy * W + ix;
    uint32_t n = 0;
    float T = 1.f, TN = 1.f;
    float Gr = 0.f, Gg = 0.f, Gb = 0.f, GA = 0.f, GD = 0.f;
    if (inside) {
        n = jb.n_contrib[p];
        TN = jb.final_T[p];
        T = TN;
        Gr = dL_drgb[p];
        Gg = dL_drgb[HW + p];
        Gb = dL_drgb[2 * HW + p];
        if (dL_dalpha) GA = dL_dalpha[p];
        if (dL_ddepth) GD = dL_ddepth[p];
    }
    const float bgr = jb.bg[0], bgg = jb.bg[1], bgb = jb.bg[2];
    // the last lane of each 16-lane row adds that row's sums to the batch
    // accumulator: components (row & 1) + 5 (row >> 1), that plus 2, and
    // 4 + 5 (row >> 1) from the even rows
    const int row = lane >> 4;
    const bool row_tail = (lane & 15) == 15;
    const int comp0 = (row & 1) + 5 * (row >> 1);
    const int comp2 = 4 + 5 * (row >> 1);
    // P = G . S - GA TN, S = (rgb, depth) blended behind the current Gaussian
    // plus the background share, G = (dL/drgb, dL/ddepth) of the pixel: then
    // dL/dalpha_i = T_i (G . c_i) - P / (1 - alpha_i), and P grows by
    // w_i (G . c_i) as the walk passes Gaussian i
    float P = TN * (Gr * bgr + Gg * bgg + Gb * bgb) - GA * TN;

    if (tid == 0) smax = 0u;
    __syncthreads();
    atomicMax(&smax, n);
    __syncthreads();
    const uint32_t nmax = smax;

    for (int64_t bend = (int64_t)nmax; bend > 0; bend -= kBwdBatch) {
        const int64_t bstart = bend - kBwdBatch > 0 ? bend - kBwdBatch : 0;
        const int nb = (int)(bend - bstart);
        __syncthreads();
        // staging at raised wave priority, as in the forward compositing: the
        // workgroup's wavefronts wait for it at the barrier (500k at 960x540:
        // 317 -> 314 us)
        __builtin_amdgcn_s_setprio(3);
        uint32_t qm = 0u;
        if (tid < nb) {
            uint32_t g = sorted_vals[s + bstart + tid];
            g = (int64_t)g < n_flat ? g : 0u;
            const GaussRec r = rec[g];
            const Staged st = stage_gaussian(r, x0, y0);
            sh0[tid] = st.s0;
            sh1[tid] = st.s1;
            sh2[tid] = st.s2;
            sh3[tid] = make_float2(st.s3.x, 1.f / r.o);
            shg[tid] = g;
#pragma unroll
            for (int c = 0; c < kG2; ++c) wacc[c][tid] = 0.f;
            // the forward's quadrant culling, so the same pairs are skipped
            qm = quadrant_mask(r, st.s0.x, st.s0.y, st.s1.y);
        }
        // bit b of qbits[c][w]: slot 64 c + b can reach quadrant w
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint64_t m = __builtin_amdgcn_ballot_w64((qm >> w) & 1u);
            if (lane == 0 && wave < kBwdBatch / 64) qbits[wave][w] = m;
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
        // each wavefront walks, last to first, the slots that can reach its quadrant
        for (int c = (nb - 1) >> 6; c >= 0; --c) {
            uint64_t m = qbits[c][wave];
            // (readfirstlane returns int: widen through uint32_t, never sign-extend)
            const uint32_t mhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(m >> 32));
            const uint32_t mlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)m);
            m = ((uint64_t)mhi << 32) | (uint64_t)mlo;
            while (m != 0ull) {
                const int bit = 63 - __builtin_clzll(m);
                m &= ~(1ull << bit);
                const int k = (c << 6) + bit;
                const uint32_t pos = (uint32_t)(bstart + k);
                const float4 s0 = sh0[k];
                const float4 s1 = sh1[k];
                const float dx = s0.x - px, dy = s0.y - py;
                const float ex = alpha_exponent(s0, s1, dx, dy);
                const bool act = inside && pos < n && ex >= kLog2AlphaMin;
                if (__ballot(act) == 0ull) continue;
                // straight-line below: lanes that do not blend the Gaussian
                // carry alpha 0 into every partial and keep T
                const float4 s2 = sh2[k];
                const float2 s3 = sh3[k];
                const float ap = fast_exp2(ex);
                const float a = fminf(ap, kAlphaMax);
                const float om = 1.f - a;
                // 1 / (1 - alpha): hardware reciprocal and one Newton step
                const float r0 = __builtin_amdgcn_rcpf(om);
                const float inv = __builtin_fmaf(__builtin_fmaf(-om, r0, 1.f), r0, r0);
                const float Ti = T * inv;
                const float am = act ? a : 0.f;
                const float w = am * Ti;
                const float Gc = Gr * s2.y + Gg * s2.z + Gb * s2.w + GD * s3.x;
                float v[kG2];
                v[6] = Gr * w;
                v[7] = Gg * w;
                v[8] = Gb * w;
                v[9] = GD * w;
                const float dLda = Ti * Gc - inv * P;
                P = __builtin_fmaf(w, Gc, P);
                T = act ? Ti : T;
                // alpha clamped at its maximum passes no gradient to the exponent.
                // Per pixel t = alpha dL/dalpha and its moments t (dx, dy, dx^2,
                // dx dy, dy^2); the conic, the 1/2 and the 1/opacity factors are
                // the same for every pixel and are applied to the tile's sums.
                const float t = (ap < kAlphaMax ? am : 0.f) * dLda;
                v[5] = t;
                v[0] = t * dx;
                v[1] = t * dy;
                v[2] = v[0] * dx;
                v[3] = v[0] * dy;
                v[4] = v[1] * dy;
                float q[3];
                wave_sums_by_row(v, q);
                if (row_tail) {
                    atomicAdd(&wacc[comp0][k], q[0]);
                    atomicAdd(&wacc[comp0 + 2][k], q[1]);
                    if ((row & 1) == 0) atomicAdd(&wacc[comp2][k], q[2]);
                }
            }
        }
        __syncthreads();
        if (tid < nb) {
            const uint32_t g = shg[tid];
            float m[kG2];
#pragma unroll
            for (int c = 0; c < kG2; ++c) m[c] = wacc[c][tid];
            // alpha = o exp(-q/2), q = A dx^2 + 2 B dx dy + C dy^2, dx = mean - pixel:
            // d alpha = alpha (-(A dx + B dy) d mu_x - (B dx + C dy) d mu_y
            //                  - dx^2 dA / 2 - dx dy dB - dy^2 dC / 2) + alpha do / o
            const float A = sh1[tid].z, B = sh1[tid].w, Cc = sh2[tid].x;
            float d[kG2];
            d[0] = -(A * m[0] + B * m[1]);
            d[1] = -(B * m[0] + Cc * m[1]);
            d[2] = -0.5f * m[2];
            d[3] = -m[3];
            d[4] = -0.5f * m[4];
            d[5] = m[5] * sh3[tid].y;
#pragma unroll
            for (int c = 6; c < kG2; ++c) d[c] = m[c];
#pragma unroll
            for (int c = 0; c < kG2; ++c)
                if (d[c] != 0.f) atomicAdd(&grads2d[(int64_t)g * kG2 + c], d[c]);
        }
    }
}

hipError_t launch_composite_bwd(const JobDev* jobs, int n_jobs, int64_t n_tiles, int64_t n_flat,
                                const GaussRec* rec, const uint32_t* sorted_vals, const uint32_t* ranges,
                                const float* dL_drgb, const float* dL_dalpha, const float* dL_ddepth, float* grads2d,
                                hipStream_t st) {
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_composite_bwd, dim3((unsigned)n_tiles), dim3(kBwdThreads), 0, st, jobs, n_jobs, rec,
                       sorted_vals, ranges, n_flat, dL_drgb, dL_dalpha, dL_ddepth, grads2d);
    return hipGetLastError();
}

// ------------------------------------------------------------------ projection adjoint

namespace {

constexpr float kB0 = 0.28209479177387814f;
constexpr float kB1 = 0.4886025119029199f;
constexpr float kB2a = 1.0925484305920792f;
constexpr float kB2b = 0.31539156525252005f;
constexpr float kB2c = 0.5462742152960396f;
constexpr float kB3a = 0.5900435899266435f;
constexpr float kB3b = 2.890611442640554f;
constexpr float kB3c = 0.4570457994644658f;
constexpr float kB3d = 0.3731763325901154f;
constexpr float kB3e = 1.445305721320277f;

// Basis values Y[k] and their partial derivatives (dYx, dYy, dYz) with the
// three direction components treated as independent.
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, int deg, float* Y, float* Gx, float* Gy,
                                              float* Gz) {
    Y[0] = kB0;
    Gx[0] = Gy[0] = Gz[0] = 0.f;
    if (deg < 1) return;
    Y[1] = -kB1 * y; Gx[1] = 0.f; Gy[1] = -kB1; Gz[1] = 0.f;
    Y[2] = kB1 * z;  Gx[2] = 0.f; Gy[2] = 0.f;  Gz[2] = kB1;
    Y[3] = -kB1 * x; Gx[3] = -kB1; Gy[3] = 0.f; Gz[3] = 0.f;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kB2a * x * y;                    Gx[4] = kB2a * y;          Gy[4] = kB2a * x;          Gz[4] = 0.f;
    Y[5] = -kB2a * y * z;                   Gx[5] = 0.f;               Gy[5] = -kB2a * z;         Gz[5] = -kB2a * y;
    Y[6] = kB2b * (2.f * zz - xx - yy);     Gx[6] = -2.f * kB2b * x;   Gy[6] = -2.f * kB2b * y;   Gz[6] = 4.f * kB2b * z;
    Y[7] = -kB2a * x * z;                   Gx[7] = -kB2a * z;         Gy[7] = 0.f;               Gz[7] = -kB2a * x;
    Y[8] = kB2c * (xx - yy);                Gx[8] = 2.f * kB2c * x;    Gy[8] = -2.f * kB2c * y;   Gz[8] = 0.f;
    if (deg < 3) return;
    Y[9] = -kB3a * y * (3.f * xx - yy);
    Gx[9] = -kB3a * 6.f * x * y;  Gy[9] = -kB3a * (3.f * xx - 3.f * yy);  Gz[9] = 0.f;
    Y[10] = kB3b * x * y * z;
    Gx[10] = kB3b * y * z;  Gy[10] = kB3b * x * z;  Gz[10] = kB3b * x * y;
    Y[11] = -kB3c * y * (4.f * zz - xx - yy);
    Gx[11] = kB3c * 2.f * x * y;  Gy[11] = -kB3c * (4.f * zz - xx - 3.f * yy);  Gz[11] = -kB3c * 8.f * y * z;
    Y[12] = kB3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Gx[12] = -kB3d * 6.f * x * z;  Gy[12] = -kB3d * 6.f * y * z;  Gz[12] = kB3d * (6.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -kB3c * x * (4.f * zz - xx - yy);
    Gx[13] = -kB3c * (4.f * zz - 3.f * xx - yy);  Gy[13] = kB3c * 2.f * x * y;  Gz[13] = -kB3c * 8.f * x * z;
    Y[14] = kB3e * z * (xx - yy);
    Gx[14] = kB3e * 2.f * x * z;  Gy[14] = -kB3e * 2.f * y * z;  Gz[14] = kB3e * (xx - yy);
    Y[15] = -kB3a * x * (xx - 3.f * yy);
    Gx[15] = -kB3a * (3.f * xx - 3.f * yy);  Gy[15] = kB3a * 6.f * x * y;  Gz[15] = 0.f;
}

// Adjoint of the SH colour at unit direction (x, y, z) for degree DEG (a
// template parameter, so the 3K coefficients and their gradients stay in
// registers and move as float4 when 3K is a multiple of 4, the pointers then
// being 16-byte aligned): accumulates dL/dcoefficients into dsh (all reads
// before the writes) and returns dL/d(direction) with the components taken
// as independent.  The colour is the forward's FP32 fused sum; below the
// clamp at 0 the channel passes no gradient.
template <int DEG, bool kSet>
__device__ __forceinline__ void sh_bwd(const float* __restrict__ sh, float* __restrict__ dsh, int64_t g, float x,
                                       float y, float z, float dr, float dg, float db, float& ddx, float& ddy,
                                       float& ddz) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int N = 3 * K;
    float Y[16], Gx[16], Gy[16], Gz[16];
    sh_basis_grad(x, y, z, DEG, Y, Gx, Gy, Gz);
    float c[N], d[N];
    const float* src = sh + g * N;
    float* dst = dsh + g * N;
    if constexpr (N % 4 == 0) {
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            const float4 t = reinterpret_cast<const float4*>(src)[k];
            const float4 u = kSet ? make_float4(0.f, 0.f, 0.f, 0.f) : reinterpret_cast<const float4*>(dst)[k];
            c[4 * k] = t.x; c[4 * k + 1] = t.y; c[4 * k + 2] = t.z; c[4 * k + 3] = t.w;
            d[4 * k] = u.x; d[4 * k + 1] = u.y; d[4 * k + 2] = u.z; d[4 * k + 3] = u.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            c[k] = src[k];
            d[k] = kSet ? 0.f : dst[k];
        }
    }
    float cr = 0.f, cg = 0.f, cb = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        cr = __builtin_fmaf(Y[k], c[3 * k + 0], cr);
        cg = __builtin_fmaf(Y[k], c[3 * k + 1], cg);
        cb = __builtin_fmaf(Y[k], c[3 * k + 2], cb);
    }
    const float e0 = cr + kColorOffset > 0.f ? dr : 0.f;
    const float e1 = cg + kColorOffset > 0.f ? dg : 0.f;
    const float e2 = cb + kColorOffset > 0.f ? db : 0.f;
    ddx = 0.f;
    ddy = 0.f;
    ddz = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        d[3 * k] += e0 * Y[k];
        d[3 * k + 1] += e1 * Y[k];
        d[3 * k + 2] += e2 * Y[k];
        const float proj = e0 * c[3 * k] + e1 * c[3 * k + 1] + e2 * c[3 * k + 2];
        ddx += proj * Gx[k];
        ddy += proj * Gy[k];
        ddz += proj * Gz[k];
    }
    if constexpr (N % 4 == 0) {
#pragma unroll
        for (int k = 0; k < N / 4; ++k)
            reinterpret_cast<float4*>(dst)[k] = make_float4(d[4 * k], d[4 * k + 1], d[4 * k + 2], d[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) dst[k] = d[k];
    }
}

}  // namespace

// kSet: the gradients are written (=) rather than added, zeros included for
// Gaussians that reach no tile, so the caller need not clear them first.
template <bool kSet>
__global__ void __launch_bounds__(256) k_project_bwd(const JobDev* __restrict__ jobs, int n_jobs, int64_t n_flat,
                                                     const uint32_t* __restrict__ touched,
                                                     const float* __restrict__ grads2d, float* __restrict__ d_means,
                                                     float* __restrict__ d_log_scales, float* __restrict__ d_quats,
                                                     float* __restrict__ d_opac, float* __restrict__ d_sh) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_flat) return;
    const int j = find_job_gauss(jobs, n_jobs, (int64_t)blockIdx.x * blockDim.x);
    const JobDev& jb = jobs[j];
    const int64_t g = i - jb.gauss_base;
    if (g >= jb.n) return;
    if (touched[i] == 0u) {
        if (kSet) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                d_means[3 * g + k] = 0.f;
                d_log_scales[3 * g + k] = 0.f;
            }
            reinterpret_cast<float4*>(d_quats)[g] = make_float4(0.f, 0.f, 0.f, 0.f);
            d_opac[g] = 0.f;
            const int n_sh = 3 * (jb.sh_degree + 1) * (jb.sh_degree + 1);
            float* dst = d_sh + g * n_sh;
            if (n_sh % 4 == 0) {
                for (int k = 0; k < n_sh / 4; ++k) reinterpret_cast<float4*>(dst)[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                for (int k = 0; k < n_sh; ++k) dst[k] = 0.f;
            }
        }
        return;
    }
    // the 10 partials as five float2 (40-byte records, 8-byte aligned)
    const float2* G2 = reinterpret_cast<const float2*>(grads2d + i * kG2);
    const float2 p01 = G2[0], p23 = G2[1], p45 = G2[2], p67 = G2[3], p89 = G2[4];
    const double du = p01.x, dv = p01.y, dA = p23.x, dB = p23.y, dC = p45.x;
    const float dop = p45.y, dr = p67.x, dgc = p67.y, db = p89.x;
    const double dzo = p89.y;
    const double* R = jb.R;

    // ---- recompute the forward quantities (FP64 geometry)
    const double mx = jb.means[3 * g], my = jb.means[3 * g + 1], mz = jb.means[3 * g + 2];
    const double x = ((R[0] * mx + R[1] * my) + R[2] * mz) + jb.t[0];
    const double y = ((R[3] * mx + R[4] * my) + R[5] * mz) + jb.t[1];
    const double z = ((R[6] * mx + R[7] * my) + R[8] * mz) + jb.t[2];
    const double gx = x / z, gy = y / z;
    const float4 qf = reinterpret_cast<const float4*>(jb.quats)[g];
    const double qw = qf.x, qx = qf.y, qy = qf.z, qz = qf.w;
    const double qn = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    const double sq = 2.0 / qn;
    double Qm[9];
    Qm[0] = -(qy * qy + qz * qz); Qm[1] = qx * qy - qw * qz; Qm[2] = qx * qz + qw * qy;
    Qm[3] = qx * qy + qw * qz;    Qm[4] = -(qx * qx + qz * qz); Qm[5] = qy * qz - qw * qx;
    Qm[6] = qx * qz - qw * qy;    Qm[7] = qy * qz + qw * qx; Qm[8] = -(qx * qx + qy * qy);
    double Rq[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rq[k] = ((k % 4) == 0 ? 1.0 : 0.0) + sq * Qm[k];
    double sc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) sc[k] = exp((double)jb.log_scales[3 * g + k]);
    double M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * sc[c];
    double Sig[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Sig[3 * a + b] = M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];
    const double j00 = jb.fx / z, j11 = jb.fy / z, j02 = -j00 * gx, j12 = -j11 * gy;
    double T0[3], T1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T0[k] = j00 * R[k] + j02 * R[6 + k];
        T1[k] = j11 * R[3 + k] + j12 * R[6 + k];
    }
    double ST0[3], ST1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ST0[k] = Sig[3 * k] * T0[0] + Sig[3 * k + 1] * T0[1] + Sig[3 * k + 2] * T0[2];
        ST1[k] = Sig[3 * k] * T1[0] + Sig[3 * k + 1] * T1[1] + Sig[3 * k + 2] * T1[2];
    }
    const double a = T0[0] * ST0[0] + T0[1] * ST0[1] + T0[2] * ST0[2] + jb.dilation;
    const double b = T0[0] * ST1[0] + T0[1] * ST1[1] + T0[2] * ST1[2];
    const double c = T1[0] * ST1[0] + T1[1] * ST1[1] + T1[2] * ST1[2] + jb.dilation;
    const double det = a * c - b * b;
    const double id = 1.0 / det, id2 = id * id;

    // ---- conic (A, B, C) = (c, -b, a) / det
    const double da = dA * (-c * c * id2) + dB * (b * c * id2) + dC * (-b * b * id2);
    const double dbb = dA * (2.0 * b * c * id2) + dB * (-id - 2.0 * b * b * id2) + dC * (2.0 * a * b * id2);
    const double dc = dA * (-b * b * id2) + dB * (a * b * id2) + dC * (-a * a * id2);

    // ---- Sigma' = Tm Sigma Tm^T
    double dSig[9];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) dSig[3 * k + l] = da * T0[k] * T0[l] + dbb * T0[k] * T1[l] + dc * T1[k] * T1[l];
    double dT0[3], dT1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dT0[k] = 2.0 * da * ST0[k] + dbb * ST1[k];
        dT1[k] = 2.0 * dc * ST1[k] + dbb * ST0[k];
    }
    // ---- Tm = J R_wc
    double dJ0[3], dJ1[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        dJ0[l] = dT0[0] * R[3 * l] + dT0[1] * R[3 * l + 1] + dT0[2] * R[3 * l + 2];
        dJ1[l] = dT1[0] * R[3 * l] + dT1[1] * R[3 * l + 1] + dT1[2] * R[3 * l + 2];
    }
    double dgx = jb.fx * du - dJ0[2] * j00;
    double dgy = jb.fy * dv - dJ1[2] * j11;
    const double dj00 = dJ0[0] - dJ0[2] * gx;
    const double dj11 = dJ1[1] - dJ1[2] * gy;
    const double iz2 = 1.0 / (z * z);
    double dzv = dzo - dj00 * jb.fx * iz2 - dj11 * jb.fy * iz2;
    const double dxv = dgx / z, dyv = dgy / z;
    dzv -= (dgx * x + dgy * y) * iz2;
    double dm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) dm[k] = R[k] * dxv + R[3 + k] * dyv + R[6 + k] * dzv;

    // ---- Sigma = M M^T, M = Rq diag(s)
    double dM[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += (dSig[3 * r + k] + dSig[3 * k + r]) * M[3 * k + cc];
            dM[3 * r + cc] = acc;
        }
    double dRq[9], dls[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        double ds = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            dRq[3 * r + cc] = dM[3 * r + cc] * sc[cc];
            ds += dM[3 * r + cc] * Rq[3 * r + cc];
        }
        dls[cc] = ds * sc[cc];
    }
    // ---- Rq = I + sq Q(q), sq = 2/|q|^2
    double dRQ = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) dRQ += dRq[k] * Qm[k];
    const double qv[4] = {qw, qx, qy, qz};
    // dQ/dq_k for k = w, x, y, z, row major 3x3
    const double dQw[9] = {0, -qz, qy, qz, 0, -qx, -qy, qx, 0};
    const double dQx[9] = {0, qy, qz, qy, -2 * qx, -qw, qz, qw, -2 * qx};
    const double dQy[9] = {-2 * qy, qx, qw, qx, 0, qz, -qw, qz, -2 * qy};
    const double dQz[9] = {-2 * qz, -qw, qx, qw, -2 * qz, qy, qx, qy, 0};
    const double* dQ[4] = {dQw, dQx, dQy, dQz};
    double dq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double acc = -2.0 * sq * qv[k] / qn * dRQ;
#pragma unroll
        for (int e = 0; e < 9; ++e) acc += sq * dRq[e] * dQ[k][e];
        dq[k] = acc;
    }

    // ---- colour: SH at the view direction d = (mean - centre) / |mean - centre|,
    // recomputed as the forward does (same reciprocal, same fused order), so
    // the clamp decision at 0 repeats the forward's
    const double c0 = -((R[0] * jb.t[0] + R[3] * jb.t[1]) + R[6] * jb.t[2]);
    const double c1 = -((R[1] * jb.t[0] + R[4] * jb.t[1]) + R[7] * jb.t[2]);
    const double c2 = -((R[2] * jb.t[0] + R[5] * jb.t[1]) + R[8] * jb.t[2]);
    const double wx = mx - c0, wy = my - c1, wz = mz - c2;
    const double len = sqrt((wx * wx + wy * wy) + wz * wz);
    const double ilen = len > 0.0 ? 1.0 / len : 0.0;
    const float ux = (float)(wx * ilen), uy = (float)(wy * ilen), uz = (float)(wz * ilen);
    float ddx, ddy, ddz;
    switch (jb.sh_degree) {
        case 0: sh_bwd<0, kSet>(jb.sh, d_sh, g, ux, uy, uz, dr, dgc, db, ddx, ddy, ddz); break;
        case 1: sh_bwd<1, kSet>(jb.sh, d_sh, g, ux, uy, uz, dr, dgc, db, ddx, ddy, ddz); break;
        case 2: sh_bwd<2, kSet>(jb.sh, d_sh, g, ux, uy, uz, dr, dgc, db, ddx, ddy, ddz); break;
        default: sh_bwd<3, kSet>(jb.sh, d_sh, g, ux, uy, uz, dr, dgc, db, ddx, ddy, ddz); break;
    }
    const float dot = ux * ddx + uy * ddy + uz * ddz;
    const float il = (float)ilen;
    dm[0] += (ddx - ux * dot) * il;
    dm[1] += (ddy - uy * dot) * il;
    dm[2] += (ddz - uz * dot) * il;

    // ---- opacity
    const float lo = jb.opac[g];
    const float o = 1.f / (1.f + __expf(-lo));

    // read every accumulator (none when writing), then write them
    const float pm0 = kSet ? 0.f : d_means[3 * g], pm1 = kSet ? 0.f : d_means[3 * g + 1],
                pm2 = kSet ? 0.f : d_means[3 * g + 2];
    const float ps0 = kSet ? 0.f : d_log_scales[3 * g], ps1 = kSet ? 0.f : d_log_scales[3 * g + 1],
                ps2 = kSet ? 0.f : d_log_scales[3 * g + 2];
    const float4 pq = kSet ? make_float4(0.f, 0.f, 0.f, 0.f) : reinterpret_cast<const float4*>(d_quats)[g];
    const float po = kSet ? 0.f : d_opac[g];
    d_means[3 * g] = pm0 + (float)dm[0];
    d_means[3 * g + 1] = pm1 + (float)dm[1];
    d_means[3 * g + 2] = pm2 + (float)dm[2];
    d_log_scales[3 * g] = ps0 + (float)dls[0];
    d_log_scales[3 * g + 1] = ps1 + (float)dls[1];
    d_log_scales[3 * g + 2] = ps2 + (float)dls[2];
    reinterpret_cast<float4*>(d_quats)[g] =
        make_float4(pq.x + (float)dq[0], pq.y + (float)dq[1], pq.z + (float)dq[2], pq.w + (float)dq[3]);
    d_opac[g] = po + dop * o * (1.f - o);
}

hipError_t launch_project_bwd(const JobDev* jobs, int n_jobs, int64_t n_flat, const uint32_t* touched,
                              const float* grads2d, float* d_means, float* d_log_scales, float* d_quats,
                              float* d_opac, float* d_sh, bool overwrite, hipStream_t st) {
    if (n_flat == 0) return hipSuccess;
    const dim3 grid((unsigned)((n_flat + 255) / 256));
    if (overwrite)
        hipLaunchKernelGGL(k_project_bwd<true>, grid, dim3(256), 0, st, jobs, n_jobs, n_flat, touched, grads2d,
                           d_means, d_log_scales, d_quats, d_opac, d_sh);
    else
        hipLaunchKernelGGL(k_project_bwd<false>, grid, dim3(256), 0, st, jobs, n_jobs, n_flat, touched, grads2d,
                           d_means, d_log_scales, d_quats, d_opac, d_sh);
    return hipGetLastError();
}

}  // namespace gs
