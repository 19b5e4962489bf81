// Device radix sort and scan for the binning stage.
//
// The per-tile depth order (3DGS^3 Sec. 3: the 2D Gaussians are depth-sorted)
// is produced by two stable LSD sorts instead of one sort of 64-bit
// (tile, depth) keys: first the Gaussians by their 32-bit depth key, then the
// (tile, Gaussian) pairs, emitted in that depth order, by tile id.  A stable
// sort by tile of a sequence already ordered by (depth, index) yields the
// (tile, depth, index) order of the 64-bit keys, while the expensive sort over
// all pairs needs only ceil(log2 tiles) bits (one 11-bit pass at 960x540).
//
// Each pass is reduce-then-scan with three kernels: a per-block digit
// histogram, a scan of every digit's counts over the blocks, and a stable
// scatter.  The scatter ranks equal digits within a wavefront with 64-bit
// ballots (one ballot per digit bit gives the mask of lanes holding the same
// digit), keeps per-wave running counts in LDS, and so never needs atomics.
#include "gs_kernels.hpp"

namespace gs {

namespace {

__device__ __forceinline__ int64_t dev_count(DevCount n) {
    if (n.dev_count == nullptr) return n.cap;
    const int64_t c = (int64_t)*n.dev_count;
    return c < n.cap ? c : n.cap;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over a block of NW wavefronts.
// `scratch` holds NW + 1 words.  Ends with a barrier so scratch can be reused.
template <int NW>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* scratch, uint32_t& total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const uint32_t w = lane < NW ? scratch[lane] : 0u;
        const uint32_t wi = wave_incl_scan(w);
        if (lane < NW) scratch[lane] = wi - w;
        if (lane == NW - 1) scratch[NW] = wi;
    }
    __syncthreads();
    const uint32_t res = incl - v + scratch[wave];
    total = scratch[NW];
    __syncthreads();
    return res;
}

}  // namespace

__global__ void __launch_bounds__(kRsThreads) k_rs_upsweep(const uint32_t* __restrict__ keys, DevCount n, int shift,
                                                           int bits, uint32_t* __restrict__ hist, int64_t nblk_cap) {
    __shared__ uint32_t h[kRsMaxBins];
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + kRsTile - 1) / kRsTile;
    if ((int64_t)blockIdx.x >= nblk) return;
    const int bins = 1 << bits;
    const uint32_t mask = (uint32_t)bins - 1u;
    for (int b = threadIdx.x; b < bins; b += kRsThreads) h[b] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t idx = base + (int64_t)r * kRsThreads + threadIdx.x;
        if (idx < cnt) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < bins; b += kRsThreads) hist[(int64_t)b * nblk_cap + blockIdx.x] = h[b];
}

// One workgroup per digit: exclusive prefix of the digit's per-block counts
// in place, digit total to totals[digit].
__global__ void __launch_bounds__(256) k_rs_scan_bins(uint32_t* __restrict__ hist, uint32_t* __restrict__ totals,
                                                      DevCount n, int64_t nblk_cap) {
    __shared__ uint32_t scratch[8];
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + kRsTile - 1) / kRsTile;
    uint32_t* row = hist + (int64_t)blockIdx.x * nblk_cap;
    uint32_t carry = 0;
    constexpr int kPer = 8;
    for (int64_t base = 0; base < nblk; base += 256 * kPer) {
        uint32_t v[kPer];
        uint32_t sum = 0;
        const int64_t first = base + (int64_t)threadIdx.x * kPer;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            v[k] = (first + k < nblk) ? row[first + k] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t run = block_excl_scan<4>(sum, scratch, tot) + carry;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (first + k < nblk) row[first + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(1024) k_rs_scan_totals(const uint32_t* __restrict__ totals,
                                                         uint32_t* __restrict__ bin_start, int bins) {
    __shared__ uint32_t scratch[17];
    const int b0 = threadIdx.x * 2;
    const uint32_t v0 = b0 < bins ? totals[b0] : 0u;
    const uint32_t v1 = b0 + 1 < bins ? totals[b0 + 1] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<16>(v0 + v1, scratch, tot);
    if (b0 < bins) bin_start[b0] = ex;
    if (b0 + 1 < bins) bin_start[b0 + 1] = ex + v0;
}

__global__ void __launch_bounds__(kRsThreads) k_rs_downsweep(const uint32_t* __restrict__ keys_in,
                                                             const uint32_t* __restrict__ vals_in,
                                                             uint32_t* __restrict__ keys_out,
                                                             uint32_t* __restrict__ vals_out, DevCount n, int shift,
                                                             int bits, const uint32_t* __restrict__ hist,
                                                             const uint32_t* __restrict__ bin_start,
                                                             int64_t nblk_cap) {
    constexpr int kWaves = kRsThreads / 64;
    __shared__ uint32_t wcnt[kWaves * kRsMaxBins];
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + kRsTile - 1) / kRsTile;
    if ((int64_t)blockIdx.x >= nblk) return;
    const int bins = 1 << bits;
    const uint32_t mask = (uint32_t)bins - 1u;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t* my = wcnt + wave * kRsMaxBins;

    for (int b = threadIdx.x; b < kWaves * bins; b += kRsThreads) wcnt[(b / bins) * kRsMaxBins + (b % bins)] = 0u;
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)wave * (kRsItems * 64);
    uint32_t key[kRsItems];
    uint64_t peers[kRsItems];
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < cnt;
        key[r] = valid ? keys_in[idx] : 0u;
        const uint32_t d = (key[r] >> shift) & mask;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        peers[r] = valid ? m : 0ull;
        if (valid && (m & lt_mask) == 0ull) my[d] += (uint32_t)__popcll(m);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < bins; b += kRsThreads) {
        uint32_t run = bin_start[b] + hist[(int64_t)b * nblk_cap + blockIdx.x];
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = wcnt[w * kRsMaxBins + b];
            wcnt[w * kRsMaxBins + b] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < cnt;
        const uint32_t d = (key[r] >> shift) & mask;
        const uint64_t m = peers[r];
        uint32_t pos = 0;
        if (valid) pos = my[d] + (uint32_t)__popcll(m & lt_mask);
        if (valid && (m & lt_mask) == 0ull) my[d] = pos + (uint32_t)__popcll(m);
        if (valid && (int64_t)pos < cnt) {
            const uint32_t val = vals_in ? vals_in[idx] : (uint32_t)idx;
            vals_out[pos] = val;
            if (keys_out) keys_out[pos] = key[r];
        }
    }
}

hipError_t radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
                      DevCount n, int shift, int bits, uint32_t* hist, uint32_t* totals, uint32_t* bin_start,
                      hipStream_t st) {
    if (n.cap == 0) return hipSuccess;
    if (bits < 1 || bits > kRsMaxBits) return hipErrorInvalidValue;
    const int64_t nblk = rs_blocks(n.cap);
    const int bins = 1 << bits;
    hipLaunchKernelGGL(k_rs_upsweep, dim3((unsigned)nblk), dim3(kRsThreads), 0, st, keys_in, n, shift, bits, hist,
                       nblk);
    hipLaunchKernelGGL(k_rs_scan_bins, dim3(bins), dim3(256), 0, st, hist, totals, n, nblk);
    hipLaunchKernelGGL(k_rs_scan_totals, dim3(1), dim3(1024), 0, st, totals, bin_start, bins);
    hipLaunchKernelGGL(k_rs_downsweep, dim3((unsigned)nblk), dim3(kRsThreads), 0, st, keys_in, vals_in, keys_out,
                       vals_out, n, shift, bits, hist, bin_start, nblk);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan

__global__ void __launch_bounds__(kRsThreads) k_scan_reduce(const uint32_t* __restrict__ order,
                                                            const uint32_t* __restrict__ touched, int64_t n,
                                                            uint32_t* __restrict__ partials) {
    __shared__ uint32_t scratch[9];
    const int64_t first = (int64_t)blockIdx.x * kRsTile + (int64_t)threadIdx.x * kRsItems;
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kRsItems; ++k)
        if (first + k < n) {
            const uint32_t o = order[first + k];
            sum += (int64_t)o < n ? touched[o] : 0u;
        }
    uint32_t tot;
    block_excl_scan<kRsThreads / 64>(sum, scratch, tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_partials(uint32_t* __restrict__ partials, int64_t nblk,
                                                        uint32_t* __restrict__ total) {
    __shared__ uint32_t scratch[17];
    uint32_t carry = 0;
    constexpr int kPer = 8;
    for (int64_t base = 0; base < nblk; base += 1024 * kPer) {
        const int64_t first = base + (int64_t)threadIdx.x * kPer;
        uint32_t v[kPer];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            v[k] = first + k < nblk ? partials[first + k] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t run = block_excl_scan<16>(sum, scratch, tot) + carry;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (first + k < nblk) partials[first + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kRsThreads) k_scan_apply(const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ touched, int64_t n,
                                                           const uint32_t* __restrict__ partials,
                                                           uint32_t* __restrict__ out) {
    __shared__ uint32_t scratch[9];
    const int64_t first = (int64_t)blockIdx.x * kRsTile + (int64_t)threadIdx.x * kRsItems;
    uint32_t v[kRsItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        const uint32_t o = first + k < n ? order[first + k] : 0xFFFFFFFFu;
        v[k] = (int64_t)o < n ? touched[o] : 0u;
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<kRsThreads / 64>(sum, scratch, tot) + partials[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        if (first + k < n) out[first + k] = run;
        run += v[k];
    }
}

hipError_t scan_gathered(const uint32_t* order, const uint32_t* touched, int64_t n, uint32_t* out,
                         uint32_t* partials, uint32_t* total, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t nblk = rs_blocks(n);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nblk), dim3(kRsThreads), 0, st, order, touched, n, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, partials, nblk, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nblk), dim3(kRsThreads), 0, st, order, touched, n, partials,
                       out);
    return hipGetLastError();
}

}  // namespace gs
