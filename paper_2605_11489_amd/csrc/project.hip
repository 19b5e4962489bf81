// Per-Gaussian projection (3DGS^3 Sec. 3): Sigma = R S S^T R^T, EWA splatting
// of the 3D Gaussian to a 2D image-space Gaussian, 3-sigma screen radius and
// tile rectangle, degree-0..3 SH colour and sigmoid opacity.
//
// One thread per Gaussian; the kernel streams 56-236 B of parameters per
// Gaussian and writes a 48 B record plus 16 B of binning data, so it is bound
// by HBM bandwidth.  Everything that decides a sort key or a tile rectangle
// (view z, the 2D mean, the 2D covariance and its largest eigenvalue, the
// radius, the rectangle) is computed in FP64 as correctly rounded IEEE
// operations in one fixed order with contraction disabled, so the keys and
// tile lists are reproducible bit for bit by any FP64 implementation that
// follows the same order.  Colour and opacity are FP32.
#include "gs_kernels.hpp"

#pragma clang fp contract(off)

namespace gs {

namespace {

// Real SH constants, sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) with the
// polynomial factors folded in (Condon-Shortley phase applied in the code).
constexpr float kSH0 = 0.28209479177387814f;    // 1/(2 sqrt(pi))
constexpr float kSH1 = 0.4886025119029199f;     // sqrt(3/(4 pi))
constexpr float kSH2a = 1.0925484305920792f;    // sqrt(15/(4 pi))
constexpr float kSH2b = 0.31539156525252005f;   // sqrt(5/(16 pi))
constexpr float kSH2c = 0.5462742152960396f;    // sqrt(15/(16 pi))
constexpr float kSH3a = 0.5900435899266435f;    // sqrt(35/(32 pi))
constexpr float kSH3b = 2.890611442640554f;     // sqrt(105/(4 pi))
constexpr float kSH3c = 0.4570457994644658f;    // sqrt(21/(32 pi))
constexpr float kSH3d = 0.3731763325901154f;    // sqrt(7/(16 pi))
constexpr float kSH3e = 1.445305721320277f;     // sqrt(105/(16 pi))

__device__ __forceinline__ void sh_basis(float x, float y, float z, int degree, float* Y) {
    Y[0] = kSH0;
    if (degree < 1) return;
    Y[1] = -kSH1 * y;
    Y[2] = kSH1 * z;
    Y[3] = -kSH1 * x;
    if (degree < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kSH2a * x * y;
    Y[5] = -kSH2a * y * z;
    Y[6] = kSH2b * (2.0f * zz - xx - yy);
    Y[7] = -kSH2a * x * z;
    Y[8] = kSH2c * (xx - yy);
    if (degree < 3) return;
    Y[9] = -kSH3a * y * (3.0f * xx - yy);
    Y[10] = kSH3b * x * y * z;
    Y[11] = -kSH3c * y * (4.0f * zz - xx - yy);
    Y[12] = kSH3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -kSH3c * x * (4.0f * zz - xx - yy);
    Y[14] = kSH3e * z * (xx - yy);
    Y[15] = -kSH3a * x * (xx - 3.0f * yy);
}

// Colour (without the +0.5 offset) from degree-DEG SH at unit direction d.
// DEG is a template parameter so every coefficient index is a constant and
// the coefficients stay in registers; 3K floats are read as float4 when 3K is
// a multiple of 4 (K = 4 or 16), which the host checks is 16-byte aligned.
template <int DEG>
__device__ __forceinline__ void sh_color(const float* __restrict__ sh, int64_t g, float x, float y, float z,
                                         float& r, float& gg, float& b) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int N = 3 * K;
    float Y[16];
    sh_basis(x, y, z, DEG, Y);
    float c[N];
    const float* src = sh + g * N;
    if constexpr (N % 4 == 0) {
        const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            const float4 t = s4[k];
            c[4 * k + 0] = t.x;
            c[4 * k + 1] = t.y;
            c[4 * k + 2] = t.z;
            c[4 * k + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) c[k] = src[k];
    }
    r = 0.f;
    gg = 0.f;
    b = 0.f;
    // colour is FP32 and not part of any key: fused multiply-adds
#pragma unroll
    for (int k = 0; k < K; ++k) {
        r = __builtin_fmaf(Y[k], c[3 * k + 0], r);
        gg = __builtin_fmaf(Y[k], c[3 * k + 1], gg);
        b = __builtin_fmaf(Y[k], c[3 * k + 2], b);
    }
}

}  // namespace

// kNormals: also write the camera-facing normal (a separate instantiation, so
// the plain projection keeps its register budget and occupancy).
// kOne: a single frame whose descriptor `one` arrives as a kernel argument;
// the first workgroup also writes it to the job table (jobs[0]) for the
// kernels after this one and clears the frame's n_zero counter words, which
// saves the frame the upload launch.  Otherwise the table is already on the
// device.
template <bool kNormals, bool kOne>
__global__ void __launch_bounds__(256) k_project(const JobDev* __restrict__ jobs, const JobDev one, int n_jobs,
                                                 int64_t n_flat, GaussRec* __restrict__ rec,
                                                 uint32_t* __restrict__ zkey, uint32_t* __restrict__ rect,
                                                 uint32_t* __restrict__ touched, float4* __restrict__ nrm,
                                                 JobDev* __restrict__ table, uint32_t* __restrict__ zero, int n_zero) {
    if (kOne && blockIdx.x == 0) {
        if (threadIdx.x == 0) table[0] = one;
        for (int w = threadIdx.x; w < n_zero; w += blockDim.x) zero[w] = 0u;
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_flat) return;
    const JobDev* jbp;
    if constexpr (kOne) {
        jbp = &one;
    } else {
        jbp = &jobs[find_job_gauss(jobs, n_jobs, (int64_t)blockIdx.x * blockDim.x)];
    }
    const JobDev& jb = *jbp;
    const int64_t g = i - jb.gauss_base;

    bool valid = g < jb.n;
    if (!valid) {
        zkey[i] = kCulledKey;
        touched[i] = 0;
        rect[i] = kEmptyRect;
        return;
    }
    const double* R = jb.R;
    const double mx = (double)jb.means[3 * g + 0];
    const double my = (double)jb.means[3 * g + 1];
    const double mz = (double)jb.means[3 * g + 2];

    // view-space position ((r0 mx + r1 my) + r2 mz) + t
    const double x = ((R[0] * mx + R[1] * my) + R[2] * mz) + jb.t[0];
    const double y = ((R[3] * mx + R[4] * my) + R[5] * mz) + jb.t[1];
    const double z = ((R[6] * mx + R[7] * my) + R[8] * mz) + jb.t[2];
    valid = z >= jb.near_z;
    const double zs = valid ? z : 1.0;
    const double gx = x / zs;
    const double gy = y / zs;
    const double limx = kGuard * ((0.5 * (double)jb.width) / jb.fx);
    const double limy = kGuard * ((0.5 * (double)jb.height) / jb.fy);
    valid = valid && !((gx < -limx) || (gx > limx) || (gy < -limy) || (gy > limy));

    // R(q) from a not necessarily unit quaternion: I + s Q(q), s = 2/|q|^2
    const float4 qf = reinterpret_cast<const float4*>(jb.quats)[g];
    const double qw = qf.x, qx = qf.y, qy = qf.z, qz = qf.w;
    const double qn = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    valid = valid && (qn > 0.0);
    const double s = 2.0 / (qn > 0.0 ? qn : 1.0);
    double Rq[9];
    Rq[0] = 1.0 - s * (qy * qy + qz * qz);
    Rq[1] = s * (qx * qy - qw * qz);
    Rq[2] = s * (qx * qz + qw * qy);
    Rq[3] = s * (qx * qy + qw * qz);
    Rq[4] = 1.0 - s * (qx * qx + qz * qz);
    Rq[5] = s * (qy * qz - qw * qx);
    Rq[6] = s * (qx * qz - qw * qy);
    Rq[7] = s * (qy * qz + qw * qx);
    Rq[8] = 1.0 - s * (qx * qx + qy * qy);

    // surface normal (computed here so R(q) need not stay live): the
    // shortest axis (first on ties of the float32 log-scales), a column of
    // R(q), in camera axes, facing the camera
    float4 nf = make_float4(0.f, 0.f, 0.f, 0.f);
    if (kNormals) {
        const float l0 = jb.log_scales[3 * g + 0], l1 = jb.log_scales[3 * g + 1], l2 = jb.log_scales[3 * g + 2];
        int k = l1 < l0 ? 1 : 0;
        if (l2 < (k ? l1 : l0)) k = 2;
        // (selects, not a dynamic index into a register array)
        const double n0 = k == 0 ? Rq[0] : (k == 1 ? Rq[1] : Rq[2]);
        const double n1 = k == 0 ? Rq[3] : (k == 1 ? Rq[4] : Rq[5]);
        const double n2 = k == 0 ? Rq[6] : (k == 1 ? Rq[7] : Rq[8]);
        double nc[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) nc[a] = (R[3 * a] * n0 + R[3 * a + 1] * n1) + R[3 * a + 2] * n2;
        const bool away = ((nc[0] * x + nc[1] * y) + nc[2] * z) > 0.0;
        const double sg = away ? -1.0 : 1.0;
        nf = make_float4((float)(sg * nc[0]), (float)(sg * nc[1]), (float)(sg * nc[2]), 0.0f);
    }

    // Sigma = M M^T with M = R diag(exp(log_scale))
    const double s0 = exp((double)jb.log_scales[3 * g + 0]);
    const double s1 = exp((double)jb.log_scales[3 * g + 1]);
    const double s2 = exp((double)jb.log_scales[3 * g + 2]);
    double M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        M[3 * r + 0] = Rq[3 * r + 0] * s0;
        M[3 * r + 1] = Rq[3 * r + 1] * s1;
        M[3 * r + 2] = Rq[3 * r + 2] * s2;
    }
    double Sig[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            Sig[3 * a + b] = (M[3 * a + 0] * M[3 * b + 0] + M[3 * a + 1] * M[3 * b + 1]) + M[3 * a + 2] * M[3 * b + 2];

    // EWA: Jacobian of the pinhole map at the mean, Tm = J R_wc, Sigma' = Tm Sigma Tm^T
    const double j00 = jb.fx / zs;
    const double j11 = jb.fy / zs;
    const double j02 = -(j00 * gx);
    const double j12 = -(j11 * gy);
    double Tm[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Tm[k] = j00 * R[k] + j02 * R[6 + k];
        Tm[3 + k] = j11 * R[3 + k] + j12 * R[6 + k];
    }
    double U[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            U[3 * r + k] = (Tm[3 * r + 0] * Sig[k] + Tm[3 * r + 1] * Sig[3 + k]) + Tm[3 * r + 2] * Sig[6 + k];
    const double ca = ((U[0] * Tm[0] + U[1] * Tm[1]) + U[2] * Tm[2]) + jb.dilation;
    const double cb = (U[0] * Tm[3] + U[1] * Tm[4]) + U[2] * Tm[5];
    const double cc = ((U[3] * Tm[3] + U[4] * Tm[4]) + U[5] * Tm[5]) + jb.dilation;
    const double det = ca * cc - cb * cb;
    valid = valid && (det > 0.0);
    if (!valid) {
        zkey[i] = kCulledKey;
        touched[i] = 0;
        rect[i] = kEmptyRect;
        return;
    }
    const double mid = 0.5 * (ca + cc);
    const double lam = mid + sqrt(fmax(0.0, mid * mid - det));
    const double radius = ceil(kSigmaCut * sqrt(fmax(lam, 0.0)));
    const double u = jb.fx * gx + jb.cx;
    const double v = jb.fy * gy + jb.cy;
    double tx0 = fmax(floor((u - radius) / (double)kTile), 0.0);
    double tx1 = fmin(floor((u + radius) / (double)kTile), (double)(jb.tiles_x - 1));
    double ty0 = fmax(floor((v - radius) / (double)kTile), 0.0);
    double ty1 = fmin(floor((v + radius) / (double)kTile), (double)(jb.tiles_y - 1));
    const float lo = jb.opac[g];
    const float opacity = 1.0f / (1.0f + __expf(-lo));
    if (jb.overlap == kOverlapOpacity || jb.overlap == kOverlapEllipse) {
        // alpha' = o exp(-q/2) >= 1/255 only inside q <= Q = 2 ln(255 o); its
        // bounding box has half-widths sqrt(Q Sigma'_xx), sqrt(Q Sigma'_yy).
        // Margins (0.1 % + 1e-3 on Q, 0.1 % + 0.02 px on the half-widths) and
        // the conditioning limit are those of the compositing's quadrant cull,
        // which bound the float32 exponent's error far below them.
        const double Q = 2.0 * log(255.0 * (double)opacity);
        if (Q < -1e-3) {
            tx1 = tx0 - 1.0;   // never reaches 1/255: no tiles
        } else if (det > 4e-3 * ca * cc) {
            const double Qm = fmax(Q, 0.0) * 1.001 + 1e-3;
            const double xe = sqrt(Qm * ca) * 1.001 + 0.02;
            const double ye = sqrt(Qm * cc) * 1.001 + 0.02;
            tx0 = fmax(tx0, floor((u - xe) / (double)kTile));
            tx1 = fmin(tx1, floor((u + xe) / (double)kTile));
            ty0 = fmax(ty0, floor((v - ye) / (double)kTile));
            ty1 = fmin(ty1, floor((v + ye) / (double)kTile));
        }
    }
    bool nonempty = (tx0 <= tx1) && (ty0 <= ty1);
    // kOverlapEllipse: of the box's tiles only those whose pixel centres the
    // ellipse can reach, counted row by row from the record's own values
    uint32_t ntiles = nonempty ? (uint32_t)(((int)tx1 - (int)tx0 + 1) * ((int)ty1 - (int)ty0 + 1)) : 0u;
    if (nonempty && jb.overlap == kOverlapEllipse) {
        const double idet0 = 1.0 / det;
        const EllipseCover ec = ellipse_cover(u, v, (float)(cc * idet0), (float)(-cb * idet0), (float)(ca * idet0),
                                              opacity);
        ntiles = 0u;
        for (int ty = (int)ty0; ty <= (int)ty1; ++ty) {
            int c0, c1;
            ellipse_row_span(ec, ty, (int)tx0, (int)tx1, c0, c1);
            ntiles += c1 >= c0 ? (uint32_t)(c1 - c0 + 1) : 0u;
        }
        nonempty = ntiles > 0u;
    }

    const float zf = (float)z;
    zkey[i] = nonempty ? __float_as_uint(zf) : kCulledKey;
    if (!nonempty) {
        touched[i] = 0;
        rect[i] = kEmptyRect;
        return;
    }
    const int ix0 = (int)tx0, ix1 = (int)tx1, iy0 = (int)ty0, iy1 = (int)ty1;
    rect[i] = (uint32_t)ix0 | ((uint32_t)iy0 << 8) | ((uint32_t)ix1 << 16) | ((uint32_t)iy1 << 24);
    touched[i] = ntiles;

    // colour: one view direction per Gaussian, from the camera centre -R^T t
    const double c0 = -((R[0] * jb.t[0] + R[3] * jb.t[1]) + R[6] * jb.t[2]);
    const double c1 = -((R[1] * jb.t[0] + R[4] * jb.t[1]) + R[7] * jb.t[2]);
    const double c2 = -((R[2] * jb.t[0] + R[5] * jb.t[1]) + R[8] * jb.t[2]);
    const double dxw = mx - c0, dyw = my - c1, dzw = mz - c2;
    const double dl = sqrt((dxw * dxw + dyw * dyw) + dzw * dzw);
    const double il = dl > 0.0 ? 1.0 / dl : 0.0;
    const float dx = (float)(dxw * il), dy = (float)(dyw * il), dz = (float)(dzw * il);
    float cr, cg, cbl;
    switch (jb.sh_degree) {
        case 0: sh_color<0>(jb.sh, g, dx, dy, dz, cr, cg, cbl); break;
        case 1: sh_color<1>(jb.sh, g, dx, dy, dz, cr, cg, cbl); break;
        case 2: sh_color<2>(jb.sh, g, dx, dy, dz, cr, cg, cbl); break;
        default: sh_color<3>(jb.sh, g, dx, dy, dz, cr, cg, cbl); break;
    }
    GaussRec r;
    r.u = u;
    r.v = v;
    // the FP32 conic from one FP64 reciprocal (no sort key depends on it; the
    // ellipse overlap mode decides tiles from exactly these values)
    const double idet = 1.0 / det;
    r.A = (float)(cc * idet);
    r.B = (float)(-cb * idet);
    r.C = (float)(ca * idet);
    r.o = opacity;
    r.r = fmaxf(cr + kColorOffset, 0.0f);
    r.g = fmaxf(cg + kColorOffset, 0.0f);
    r.b = fmaxf(cbl + kColorOffset, 0.0f);
    r.z = zf;
    rec[i] = r;
    if (kNormals) nrm[i] = nf;
}

hipError_t launch_project(const JobDev* jobs, int n_jobs, int64_t n_flat, GaussRec* rec, uint32_t* zkey,
                          uint32_t* rect, uint32_t* touched, float4* nrm, hipStream_t st) {
    if (n_flat == 0) return hipSuccess;
    const int64_t blocks = (n_flat + 255) / 256;
    const JobDev none{};
    if (nrm)
        hipLaunchKernelGGL((k_project<true, false>), dim3((unsigned)blocks), dim3(256), 0, st, jobs, none, n_jobs,
                           n_flat, rec, zkey, rect, touched, nrm, nullptr, nullptr, 0);
    else
        hipLaunchKernelGGL((k_project<false, false>), dim3((unsigned)blocks), dim3(256), 0, st, jobs, none, n_jobs,
                           n_flat, rec, zkey, rect, touched, nrm, nullptr, nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_project_one(const JobDev& one, JobDev* table, uint32_t* zero, int n_zero, int64_t n_flat,
                              GaussRec* rec, uint32_t* zkey, uint32_t* rect, uint32_t* touched, float4* nrm,
                              hipStream_t st) {
    // (one workgroup at least, so the table and the counters are written)
    const int64_t blocks = n_flat > 0 ? (n_flat + 255) / 256 : 1;
    if (nrm)
        hipLaunchKernelGGL((k_project<true, true>), dim3((unsigned)blocks), dim3(256), 0, st, table, one, 1, n_flat,
                           rec, zkey, rect, touched, nrm, table, zero, n_zero);
    else
        hipLaunchKernelGGL((k_project<false, true>), dim3((unsigned)blocks), dim3(256), 0, st, table, one, 1, n_flat,
                           rec, zkey, rect, touched, nrm, table, zero, n_zero);
    return hipGetLastError();
}

}  // namespace gs
