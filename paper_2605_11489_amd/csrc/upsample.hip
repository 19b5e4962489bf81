// Gradient-aware interpolation of the low-resolution image to S x S times its
// pixels (3DGS^3 Sec. 4.1, Eq. 5-7) with a fixed least-squares matrix M.
//
// For pixel (x0, y0), the 27 inputs are the image values, x-derivatives and
// y-derivatives at the 3x3 block of pixel centres around it (node (i, j) at
// offset (i, j), n = 3 (j + 1) + (i + 1); nodes outside the image take the
// nearest edge pixel).  The S x S high-resolution pixels covering (x0, y0),
// centred at offsets ((k + 0.5)/S - 0.5, (l + 0.5)/S - 0.5), are each one
// linear combination of the 27 (Eq. 7).  M is the least-squares fit of the
// polynomials of total degree <= 5 (21 terms; the bicubic space is
// rank-deficient on this stencil) to the 27 conditions of Eq. 5, evaluated
// at the sub-pixel centres, so every such polynomial is reproduced exactly.
// The host builds M in FP64 (Householder least squares) and passes it in the
// kernel arguments, so every coefficient is a scalar operand.
//
// One workgroup per 16 x 16 low-resolution pixels stages its tile and a
// one-pixel halo of all nine input planes in LDS; each thread writes its
// S x S block of each channel as S rows of S floats.  S^2 x 27 FMAs per pixel
// and channel against 4 S^2 bytes written: HBM-bound for S >= 2 (per
// low-resolution pixel 36 B read, 12 S^2 B written).
#include <math.h>
#include <string.h>

#include <mutex>

#include "gs_kernels.hpp"

namespace gs {

namespace {

constexpr int kUpTile = 16;
constexpr int kUpHalo = kUpTile + 2;
constexpr int kUpIn = 27;
constexpr int kUpBasis = 21;   // x^a y^b, a + b <= 5

// M with each row padded to 28 floats, so a row is seven 16-byte reads
constexpr int kUpRow = 28;

template <int S>
struct UpMatrix {
    float m[S * S][kUpRow];
};

template <int S>
__global__ void __launch_bounds__(kUpTile* kUpTile) k_upsample(const float* __restrict__ rgb,
                                                                const float* __restrict__ dcdx,
                                                                const float* __restrict__ dcdy, int W, int H,
                                                                float* __restrict__ out, UpMatrix<S> M) {
    // [plane][y][x], planes: value, d/dx, d/dy of channels 0..2
    __shared__ float tile[9][kUpHalo][kUpHalo];
    // M in LDS: its reads are broadcasts, and each coefficient serves the three channels
    __shared__ float4 sm[S * S * kUpRow / 4];
    // 1D grid over the tiles in XCD-contiguous order (halo lines stay in one L2)
    const int gx = (W + kUpTile - 1) / kUpTile, gy = (H + kUpTile - 1) / kUpTile;
    const int lt = (int)xcd_block(blockIdx.x, (int64_t)gx * gy);
    const int bx = (lt % gx) * kUpTile, by = (lt / gx) * kUpTile;
    const int64_t HW = (int64_t)W * H;
    for (int e = threadIdx.x; e < S * S * kUpRow / 4; e += kUpTile * kUpTile) {
        const float* src = &M.m[0][0] + 4 * e;
        sm[e] = make_float4(src[0], src[1], src[2], src[3]);
    }
    for (int e = threadIdx.x; e < kUpHalo * kUpHalo; e += kUpTile * kUpTile) {
        const int hy = e / kUpHalo, hx = e % kUpHalo;
        const int x = min(max(bx + hx - 1, 0), W - 1);
        const int y = min(max(by + hy - 1, 0), H - 1);
        const int64_t p = (int64_t)y * W + x;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            tile[c][hy][hx] = rgb[c * HW + p];
            tile[3 + c][hy][hx] = dcdx[c * HW + p];
            tile[6 + c][hy][hx] = dcdy[c * HW + p];
        }
    }
    __syncthreads();
    const int tx = threadIdx.x % kUpTile, ty = threadIdx.x / kUpTile;
    const int x0 = bx + tx, y0 = by + ty;
    if (x0 >= W || y0 >= H) return;
    const int64_t WS = (int64_t)W * S;
    const int64_t plane = WS * H * S;
    // the 27 inputs of the three channels (the 28th column of M is zero)
    float v[3][kUpRow];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int n = 3 * j + i;
                v[c][n] = tile[c][ty + j][tx + i];
                v[c][9 + n] = tile[3 + c][ty + j][tx + i];
                v[c][18 + n] = tile[6 + c][ty + j][tx + i];
            }
        v[c][27] = 0.f;
    }
#pragma unroll
    for (int l = 0; l < S; ++l) {
        float row[3][S];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
            for (int q4 = 0; q4 < kUpRow / 4; ++q4) {
                const float4 m = sm[((l * S + k) * kUpRow) / 4 + q4];
                const float mm[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (4 * q4 + t >= kUpIn) continue;   // padding column
                    a0 = __builtin_fmaf(mm[t], v[0][4 * q4 + t], a0);
                    a1 = __builtin_fmaf(mm[t], v[1][4 * q4 + t], a1);
                    a2 = __builtin_fmaf(mm[t], v[2][4 * q4 + t], a2);
                }
            }
            row[0][k] = a0;
            row[1][k] = a1;
            row[2][k] = a2;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float* dst = out + c * plane + ((int64_t)y0 * S + l) * WS + (int64_t)x0 * S;
            if constexpr (S == 4) {
                *reinterpret_cast<float4*>(dst) = make_float4(row[c][0], row[c][1], row[c][2], row[c][3]);
            } else if constexpr (S == 2) {
                *reinterpret_cast<float2*>(dst) = make_float2(row[c][0], row[c][1]);
            } else {
#pragma unroll
                for (int k = 0; k < S; ++k) dst[k] = row[c][k];
            }
        }
    }
}

// S = 4 on the matrix cores: Eq. 7 is a product of M (16 sub-pixels x 27
// inputs) with the inputs of the pixels.  v_mfma_f32_16x16x4f32 takes a
// 16 x 4 slice of M (lane l: row l % 16, column l / 16 of the slice), a 4 x 16
// slice of inputs (lane l: input l / 16 of the slice for column l % 16) and
// accumulates a 16 x 16 block (lane l: rows 4 (l / 16) .. + 3 of column
// l % 16).  Columns are 16 pixels of one row and channel, so lane l ends with
// output row l / 16 of pixel l % 16's 4 x 4 block: one float4 store.  Seven
// K steps cover the 27 inputs (the 28th column of M is zero).  Each
// wavefront takes 4 rows of the 16 x 16 tile.
__global__ void __launch_bounds__(kUpTile* kUpTile) k_upsample4_mfma(const float* __restrict__ rgb,
                                                                      const float* __restrict__ dcdx,
                                                                      const float* __restrict__ dcdy, int W, int H,
                                                                      float* __restrict__ out, UpMatrix<4> M) {
    __shared__ float tile[9][kUpHalo][kUpHalo];
    // 1D grid over the tiles in XCD-contiguous order (halo lines stay in one L2)
    const int gx = (W + kUpTile - 1) / kUpTile, gy = (H + kUpTile - 1) / kUpTile;
    const int lt = (int)xcd_block(blockIdx.x, (int64_t)gx * gy);
    const int bx = (lt % gx) * kUpTile, by = (lt / gx) * kUpTile;
    const int64_t HW = (int64_t)W * H;
    for (int e = threadIdx.x; e < kUpHalo * kUpHalo; e += kUpTile * kUpTile) {
        const int hy = e / kUpHalo, hx = e % kUpHalo;
        const int x = min(max(bx + hx - 1, 0), W - 1);
        const int y = min(max(by + hy - 1, 0), H - 1);
        const int64_t p = (int64_t)y * W + x;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            tile[c][hy][hx] = rgb[c * HW + p];
            tile[3 + c][hy][hx] = dcdx[c * HW + p];
            tile[6 + c][hy][hx] = dcdy[c * HW + p];
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    // this lane's slice entries of M: row col, columns 4 kk + kq
    float a[7];
#pragma unroll
    for (int kk = 0; kk < 7; ++kk) a[kk] = M.m[col][4 * kk + kq];
    __syncthreads();
    const int64_t WS = (int64_t)W * 4;
    const int64_t plane = WS * H * 4;
    const int x0 = bx + col;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ty = wave * 4 + r;
        const int y0 = by + ty;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            typedef float f4 __attribute__((ext_vector_type(4)));
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 7; ++kk) {
                const int q = 4 * kk + kq;                 // input index of this lane
                const int pl = q / 9, n = q % 9;           // plane (value, d/dx, d/dy), node
                const float b = q < kUpIn ? tile[3 * pl + c][ty + n / 3][col + n % 3] : 0.f;
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b, acc, 0, 0, 0);
            }
            if (x0 < W && y0 < H)
                *reinterpret_cast<float4*>(out + c * plane + ((int64_t)y0 * 4 + kq) * WS + (int64_t)x0 * 4) =
                    make_float4(acc[0], acc[1], acc[2], acc[3]);
        }
    }
}

// ---- host: M = E pinv(A) in FP64

void basis_row(double x, double y, int deriv, double* out) {
    int t = 0;
    for (int b = 0; b <= 5; ++b)
        for (int a = 0; a + b <= 5; ++a) {
            double v;
            if (deriv == 0)
                v = pow(x, a) * pow(y, b);
            else if (deriv == 1)
                v = a ? a * pow(x, a - 1) * pow(y, b) : 0.0;
            else
                v = b ? b * pow(x, a) * pow(y, b - 1) : 0.0;
            out[t++] = v;
        }
}

// Least-squares solution operator of A (27 x 21, full column rank) by
// Householder QR: X = pinv(A) = R^-1 Q^T, written as X[21][27].
void pinv_qr(double A[kUpIn][kUpBasis], double X[kUpBasis][kUpIn]) {
    double R[kUpIn][kUpBasis];
    double Qt[kUpIn][kUpIn];   // accumulates Q^T
    memcpy(R, A, sizeof(R));
    for (int i = 0; i < kUpIn; ++i)
        for (int j = 0; j < kUpIn; ++j) Qt[i][j] = i == j ? 1.0 : 0.0;
    for (int k = 0; k < kUpBasis; ++k) {
        double norm = 0.0;
        for (int i = k; i < kUpIn; ++i) norm += R[i][k] * R[i][k];
        norm = sqrt(norm);
        const double alpha = R[k][k] > 0 ? -norm : norm;
        double v[kUpIn] = {0};
        for (int i = k; i < kUpIn; ++i) v[i] = R[i][k];
        v[k] -= alpha;
        double vv = 0.0;
        for (int i = k; i < kUpIn; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        for (int j = 0; j < kUpBasis; ++j) {
            double d = 0.0;
            for (int i = k; i < kUpIn; ++i) d += v[i] * R[i][j];
            d = 2.0 * d / vv;
            for (int i = k; i < kUpIn; ++i) R[i][j] -= d * v[i];
        }
        for (int j = 0; j < kUpIn; ++j) {
            double d = 0.0;
            for (int i = k; i < kUpIn; ++i) d += v[i] * Qt[i][j];
            d = 2.0 * d / vv;
            for (int i = k; i < kUpIn; ++i) Qt[i][j] -= d * v[i];
        }
    }
    // X = R^-1 (first 21 rows of Q^T), back substitution column by column
    for (int col = 0; col < kUpIn; ++col)
        for (int i = kUpBasis - 1; i >= 0; --i) {
            double s = Qt[i][col];
            for (int j = i + 1; j < kUpBasis; ++j) s -= R[i][j] * X[j][col];
            X[i][col] = s / R[i][i];
        }
}

template <int S>
const UpMatrix<S>& up_matrix() {
    static UpMatrix<S> M;
    static std::once_flag once;
    std::call_once(once, [] {
        double A[kUpIn][kUpBasis];
        for (int j = -1; j <= 1; ++j)
            for (int i = -1; i <= 1; ++i) {
                const int n = 3 * (j + 1) + (i + 1);
                basis_row(i, j, 0, A[n]);
                basis_row(i, j, 1, A[9 + n]);
                basis_row(i, j, 2, A[18 + n]);
            }
        double X[kUpBasis][kUpIn];
        pinv_qr(A, X);
        for (int l = 0; l < S; ++l)
            for (int k = 0; k < S; ++k) {
                double e[kUpBasis];
                basis_row((k + 0.5) / S - 0.5, (l + 0.5) / S - 0.5, 0, e);
                for (int q = 0; q < kUpIn; ++q) {
                    double s = 0.0;
                    for (int t = 0; t < kUpBasis; ++t) s += e[t] * X[t][q];
                    M.m[l * S + k][q] = (float)s;
                }
                M.m[l * S + k][kUpIn] = 0.f;
            }
    });
    return M;
}

template <int S>
hipError_t launch_up(const float* rgb, const float* dcdx, const float* dcdy, int W, int H, float* out,
                     hipStream_t st) {
    const dim3 grid((unsigned)(((W + kUpTile - 1) / kUpTile) * ((H + kUpTile - 1) / kUpTile)));
    hipLaunchKernelGGL(k_upsample<S>, grid, dim3(kUpTile * kUpTile), 0, st, rgb, dcdx, dcdy, W, H, out,
                       up_matrix<S>());
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gradient_upsample(const float* rgb, const float* dcdx, const float* dcdy, int W, int H, int S,
                                    float* out, hipStream_t st) {
    switch (S) {
        case 1: return launch_up<1>(rgb, dcdx, dcdy, W, H, out, st);
        case 2: return launch_up<2>(rgb, dcdx, dcdy, W, H, out, st);
        case 3: return launch_up<3>(rgb, dcdx, dcdy, W, H, out, st);
        case 4: {
            const dim3 grid((unsigned)(((W + kUpTile - 1) / kUpTile) * ((H + kUpTile - 1) / kUpTile)));
            hipLaunchKernelGGL(k_upsample4_mfma, grid, dim3(kUpTile * kUpTile), 0, st, rgb, dcdx, dcdy, W, H, out,
                               up_matrix<4>());
            return hipGetLastError();
        }
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gs
