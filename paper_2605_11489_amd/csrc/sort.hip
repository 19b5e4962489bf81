// Device radix sort and scan for the binning stage.
//
// The per-tile depth order (3DGS^3 Sec. 3: the 2D Gaussians are depth-sorted)
// is produced by two stable LSD sorts instead of one sort of 64-bit
// (tile, depth) keys: first the Gaussians by their 32-bit depth key, then the
// (tile, Gaussian) pairs, emitted in that depth order, by tile id.  A stable
// sort by tile of a sequence already ordered by (depth, index) yields the
// (tile, depth, index) order of the 64-bit keys, while the sort over all
// pairs needs only ceil(log2 tiles) bits (two passes at 960x540).
//
// Each pass (digit of at most 8 bits) is reduce-then-scan:
//   1. k_rs_upsweep: per-block digit histogram (LDS atomics);
//   2. k_rs_scan: per digit, exclusive prefix of its counts over the blocks,
//      and the digit total (the scatter scans the 256 totals itself);
//   3. k_rs_downsweep: stable scatter.  Equal digits are ranked inside a
//      wavefront with one 64-bit ballot per digit bit (the AND of the
//      matching masks is the set of lanes holding the same digit), per-wave
//      running counts live in LDS, the block's elements are first placed in
//      LDS in digit order, and only then written out, so each digit's run of
//      a block leaves as one contiguous, coalesced segment.
#include "gs_kernels.hpp"

namespace gs {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

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

template <int THREADS, int ITEMS>
__global__ void __launch_bounds__(THREADS) k_rs_upsweep(const uint32_t* __restrict__ keys, DevCount n, int shift,
                                                        int bits, uint32_t* __restrict__ hist, int64_t nblk_cap) {
    constexpr int TILE = THREADS * ITEMS;
    __shared__ uint32_t h[kRsMaxBins];
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + TILE - 1) / TILE;
    if ((int64_t)blockIdx.x >= nblk) return;
    const int bins = 1 << bits;
    const uint32_t mask = (uint32_t)bins - 1u;
    if ((int)threadIdx.x < bins) h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * TILE;
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int64_t idx = base + (int64_t)r * THREADS + threadIdx.x;
        if (idx < cnt) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    if ((int)threadIdx.x < bins) hist[(int64_t)threadIdx.x * nblk_cap + blockIdx.x] = h[threadIdx.x];
}

// One workgroup per digit: exclusive prefix of the digit's per-block counts in
// place, and the digit's total.
template <int ITEMS_TILE>
__global__ void __launch_bounds__(kThreads) k_rs_scan(uint32_t* __restrict__ hist, uint32_t* __restrict__ totals,
                                                      DevCount n, int64_t nblk_cap) {
    __shared__ uint32_t scratch[kWaves + 1];
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + ITEMS_TILE - 1) / ITEMS_TILE;
    uint32_t* row = hist + (int64_t)blockIdx.x * nblk_cap;
    uint32_t carry = 0;
    constexpr int kPer = 8;
    for (int64_t b0 = 0; b0 < nblk; b0 += kThreads * kPer) {
        uint32_t v[kPer];
        uint32_t sum = 0;
        const int64_t first = b0 + (int64_t)threadIdx.x * kPer;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            v[k] = (first + k < nblk) ? row[first + k] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t run = block_excl_scan<kWaves>(sum, scratch, tot) + carry;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (first + k < nblk) row[first + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of one pass.  The digit start offsets are the exclusive scan
// of the digit totals, recomputed by every block (256 values) instead of by
// another launch.
// BITS > 0 fixes the digit width at compile time (the matching loop unrolls
// and its masks stay in scalar registers); BITS == 0 reads it from `bits`.
template <int THREADS, int ITEMS, bool V2, int BITS>
__global__ void __launch_bounds__(THREADS) k_rs_downsweep(const uint32_t* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in,
                                                          const uint32_t* __restrict__ vals2_in,
                                                          uint32_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out,
                                                          uint32_t* __restrict__ vals2_out, DevCount n, int shift,
                                                          int bits, const uint32_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ totals, int64_t nblk_cap) {
    constexpr int TILE = THREADS * ITEMS;
    constexpr int WAVES = THREADS / 64;
    __shared__ uint32_t skey[TILE];
    __shared__ uint32_t sval[TILE];
    __shared__ uint32_t sval2[V2 ? TILE : 1];
    __shared__ uint32_t wcnt[WAVES][kRsMaxBins];
    __shared__ int32_t gofs[kRsMaxBins];
    __shared__ uint32_t scratch[WAVES + 1];
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + TILE - 1) / TILE;
    if ((int64_t)blockIdx.x >= nblk) return;
    if (BITS) bits = BITS;
    const int bins = 1 << bits;
    const uint32_t mask = (uint32_t)bins - 1u;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * TILE;
    const int n_local = (int)((cnt - base) < TILE ? (cnt - base) : TILE);

    for (int e = threadIdx.x; e < WAVES * kRsMaxBins; e += THREADS) (&wcnt[0][0])[e] = 0u;
    __syncthreads();

    // phase 1: keys and values in registers, per-wave digit counts
    const int wbase = wave * 64 * ITEMS;
    uint32_t key[ITEMS], val[ITEMS], val2[ITEMS];
    uint64_t peers[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int li = wbase + r * 64 + lane;
        const bool valid = li < n_local;
        key[r] = valid ? keys_in[base + li] : 0u;
        val[r] = valid ? (vals_in ? vals_in[base + li] : (uint32_t)(base + li)) : 0u;
        if (V2) val2[r] = valid ? vals2_in[base + li] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int li = wbase + r * 64 + lane;
        const bool valid = li < n_local;
        const uint32_t d = (key[r] >> shift) & mask;
        // lanes holding the same digit: AND over the digit bits of the ballot
        // of that bit, complemented where this lane's bit is clear
        const uint64_t vm = __ballot(valid);
        uint32_t mlo = (uint32_t)vm, mhi = (uint32_t)(vm >> 32);
        const uint32_t nd = ~d;
#pragma unroll
        for (int b = 0; b < (BITS ? BITS : kRsMaxBits); ++b) {
            if (!BITS && b >= bits) break;
            const uint64_t bb = __ballot((d >> b) & 1u);
            const uint32_t sx = (uint32_t)__builtin_amdgcn_sbfe((int)nd, b, 1);   // -1 where bit b is clear
            mlo &= (uint32_t)bb ^ sx;
            mhi &= (uint32_t)(bb >> 32) ^ sx;
        }
        const uint64_t m = ((uint64_t)mhi << 32) | mlo;
        peers[r] = valid ? m : 0ull;
        if (valid && (m & lt_mask) == 0ull) wcnt[wave][d] += (uint32_t)__popcll(m);
    }
    __syncthreads();

    // phase 2: digit starts (global and block-local), per-wave running positions
    {
        const int d = threadIdx.x;
        const uint32_t td = d < bins ? totals[d] : 0u;
        uint32_t all;
        const uint32_t gstart = block_excl_scan<WAVES>(td, scratch, all);
        uint32_t c[WAVES];
        uint32_t tot_d = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            c[w] = d < bins ? wcnt[w][d] : 0u;
            tot_d += c[w];
        }
        const uint32_t lstart = block_excl_scan<WAVES>(tot_d, scratch, all);
        if (d < bins) {
            uint32_t run = lstart;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                wcnt[w][d] = run;
                run += c[w];
            }
            gofs[d] = (int32_t)(gstart + hist[(int64_t)d * nblk_cap + blockIdx.x]) - (int32_t)lstart;
        }
    }
    __syncthreads();

    // phase 3: stable local placement in LDS
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int li = wbase + r * 64 + lane;
        const bool valid = li < n_local;
        const uint32_t d = (key[r] >> shift) & mask;
        const uint64_t m = peers[r];
        uint32_t pos = 0;
        if (valid) pos = wcnt[wave][d] + (uint32_t)__popcll(m & lt_mask);
        if (valid && (m & lt_mask) == 0ull) wcnt[wave][d] = pos + (uint32_t)__popcll(m);
        if (valid && pos < (uint32_t)TILE) {
            skey[pos] = key[r];
            sval[pos] = val[r];
            if (V2) sval2[pos] = val2[r];
        }
    }
    __syncthreads();

    // phase 4: coalesced write-out, digit runs are contiguous in LDS and in memory
    for (int i = threadIdx.x; i < n_local; i += THREADS) {
        const uint32_t k = skey[i];
        const int64_t gpos = (int64_t)gofs[(k >> shift) & mask] + i;
        if (gpos >= 0 && gpos < cnt) {
            vals_out[gpos] = sval[i];
            if (V2) vals2_out[gpos] = sval2[i];
            if (keys_out) keys_out[gpos] = k;
        }
    }
}

// Large passes: 512 threads x 8 elements; small passes (depth sort of one
// frame's Gaussians): 256 x 4, so that a pass still spreads over the CUs.
constexpr int64_t kBigPass = (int64_t)4 << 20;

int64_t rs_pass_blocks(int64_t cap) {
    const int64_t tile = cap >= kBigPass ? 4096 : 1024;
    return (cap + tile - 1) / tile;
}

template <int THREADS, int ITEMS, bool V2, int BITS>
static void launch_down(const uint32_t* keys_in, const uint32_t* vals_in, const uint32_t* vals2_in,
                        uint32_t* keys_out, uint32_t* vals_out, uint32_t* vals2_out, DevCount n, int shift, int bits,
                        const uint32_t* hist, const uint32_t* totals, int64_t nblk, hipStream_t st) {
    hipLaunchKernelGGL((k_rs_downsweep<THREADS, ITEMS, V2, BITS>), dim3((unsigned)nblk), dim3(THREADS), 0, st,
                       keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift, bits, hist, totals, nblk);
}

template <int THREADS, int ITEMS, bool V2>
static void launch_pass(const uint32_t* keys_in, const uint32_t* vals_in, const uint32_t* vals2_in,
                        uint32_t* keys_out, uint32_t* vals_out, uint32_t* vals2_out, DevCount n, int shift, int bits,
                        uint32_t* hist, uint32_t* totals, hipStream_t st) {
    const int64_t nblk = rs_pass_blocks(n.cap);
    const int bins = 1 << bits;
    hipLaunchKernelGGL((k_rs_upsweep<THREADS, ITEMS>), dim3((unsigned)nblk), dim3(THREADS), 0, st, keys_in, n, shift,
                       bits, hist, nblk);
    hipLaunchKernelGGL((k_rs_scan<THREADS * ITEMS>), dim3(bins), dim3(kThreads), 0, st, hist, totals, n, nblk);
    switch (bits) {
        case 5: launch_down<THREADS, ITEMS, V2, 5>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift,
                                                    bits, hist, totals, nblk, st); break;
        case 6: launch_down<THREADS, ITEMS, V2, 6>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift,
                                                    bits, hist, totals, nblk, st); break;
        case 7: launch_down<THREADS, ITEMS, V2, 7>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift,
                                                    bits, hist, totals, nblk, st); break;
        case 8: launch_down<THREADS, ITEMS, V2, 8>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift,
                                                    bits, hist, totals, nblk, st); break;
        default: launch_down<THREADS, ITEMS, V2, 0>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n,
                                                     shift, bits, hist, totals, nblk, st); break;
    }
}

hipError_t radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, const uint32_t* vals2_in,
                      uint32_t* keys_out, uint32_t* vals_out, uint32_t* vals2_out, DevCount n, int shift, int bits,
                      uint32_t* hist, uint32_t* totals, hipStream_t st) {
    if (n.cap == 0) return hipSuccess;
    if (bits < 1 || bits > kRsMaxBits) return hipErrorInvalidValue;
    if ((vals2_in == nullptr) != (vals2_out == nullptr)) return hipErrorInvalidValue;
    const bool two = vals2_in != nullptr;
    if (n.cap >= kBigPass) {
        if (two)
            launch_pass<512, 8, true>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift, bits,
                                      hist, totals, st);
        else
            launch_pass<512, 8, false>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift, bits,
                                       hist, totals, st);
    } else {
        if (two)
            launch_pass<256, 4, true>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift, bits,
                                      hist, totals, st);
        else
            launch_pass<256, 4, false>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift, bits,
                                       hist, totals, st);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan

constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;

int64_t scan_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t* __restrict__ rects, int64_t n,
                                                          uint32_t* __restrict__ partials) {
    __shared__ uint32_t scratch[kWaves + 1];
    const int64_t first = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (first + k < n) sum += rect_tiles(rects[first + k]);
    uint32_t tot;
    block_excl_scan<kWaves>(sum, scratch, tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_partials(uint32_t* __restrict__ partials, int64_t nblk,
                                                        uint32_t* __restrict__ total) {
    __shared__ uint32_t scratch[17];
    uint32_t carry = 0;
    constexpr int kPer = 8;
    for (int64_t b0 = 0; b0 < nblk; b0 += 1024 * kPer) {
        const int64_t first = b0 + (int64_t)threadIdx.x * kPer;
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

__global__ void __launch_bounds__(kThreads) k_scan_apply(const uint32_t* __restrict__ rects, int64_t n,
                                                         const uint32_t* __restrict__ partials,
                                                         uint32_t* __restrict__ out) {
    __shared__ uint32_t scratch[kWaves + 1];
    const int64_t first = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = first + k < n ? rect_tiles(rects[first + k]) : 0u;
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<kWaves>(sum, scratch, tot) + partials[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (first + k < n) out[first + k] = run;
        run += v[k];
    }
}

hipError_t scan_rects(const uint32_t* rects, int64_t n, uint32_t* out, uint32_t* partials, uint32_t* total,
                      hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t nblk = scan_blocks(n);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nblk), dim3(kThreads), 0, st, rects, n, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, partials, nblk, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nblk), dim3(kThreads), 0, st, rects, n, partials, out);
    return hipGetLastError();
}

}  // namespace gs
