// Device radix sort and scan for the binning stage.
//
// The per-tile depth order (3DGS^3 Sec. 3: the 2D Gaussians are depth-sorted)
// is produced by two stable LSD sorts instead of one sort of 64-bit
// (tile, depth) keys: first the Gaussians by their 32-bit depth key, then the
// (tile, Gaussian) pairs, emitted in that depth order, by tile id.  A stable
// sort by tile of a sequence already ordered by (depth, index) yields the
// (tile, depth, index) order of the 64-bit keys, while the sort over all
// pairs needs only ceil(log2 tiles) bits: one pass of 11 bits at 960x540.
//
// Each pass (digit of at most 11 bits, blocks of 4096 elements, 8192 in the
// banded tile pass) is reduce-then-scan:
//   1. k_rs_upsweep: per-block digit histogram (LDS atomics), stored as one
//      contiguous row of 16-bit counts per block;
//   2. k_rs_group: blocks in groups of 16 (8 in the banded pass): per digit,
//      the exclusive prefix of the counts inside the group (in place) and the
//      group total;
//   3. k_rs_gscan: per digit, the exclusive prefix of the group totals over
//      the groups (in place) and the digit total (the scatter scans the
//      digit totals itself); passes over fewer than 4M elements do 2 and 3
//      in one launch, k_rs_groupscan;
//   4. k_rs_downsweep: stable scatter.  Each element is ranked among the
//      earlier elements of its wavefront holding the same digit by one
//      returning LDS atomic add on the wavefront's counter of that digit: the
//      LDS applies the same-address adds of one wavefront instruction in
//      lane order (measured on gfx950: no exception in 2.7e8 rows of random
//      and duplicated digits; the bit-exact sort tests rest on it too), and a
//      wavefront's rows are issued in order.  The block's elements are placed
//      in LDS in digit order and only then written out, so each digit's run
//      of a block leaves as one contiguous, coalesced segment.  When the
//      digit is a whole tile id, the digit starts and totals are the tile
//      ranges, which the first workgroup writes.
// The scatter's workgroup width is chosen apart from its block of elements
// (see kScatterThreads).  Workgroups are dealt round-robin to the eight XCDs,
// so blocks are renumbered to give each XCD a contiguous run of blocks: a
// group's blocks then share one XCD's L2.
#include "gs_kernels.hpp"

namespace gs {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
// elements per thread of a radix block: 16 (4096 per block) for every pass.
// Passes over fewer than kBigPass elements (a frame's depth sort) fold the
// block histograms in one launch (k_rs_groupscan) instead of two; 2048 per
// block there spread the depth sort over more CUs but cost more digit
// bookkeeping, and measured 2.3 us slower over 1M keys.
#ifndef GS_RS_ITEMS_BIG
#define GS_RS_ITEMS_BIG 16
#endif
#ifndef GS_RS_ITEMS_SMALL
#define GS_RS_ITEMS_SMALL 16
#endif
constexpr int kRsItemsBig = GS_RS_ITEMS_BIG;
constexpr int kRsItemsSmall = GS_RS_ITEMS_SMALL;
constexpr int64_t kBigPass = (int64_t)4 << 20;
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t dev_count(DevCount n) {
    if (n.dev_count == nullptr) return n.cap;
    const int64_t c = (int64_t)*n.dev_count;
    return c < n.cap ? c : n.cap;
}

// Logical block of workgroup b among nblk: the workgroups of XCD x = b % 8
// take the contiguous logical range that starts at x * (nblk / 8) + min(x, nblk % 8).
__device__ __forceinline__ int64_t logical_block(int64_t b, int64_t nblk) {
    const int64_t q = nblk / kXcds, r = nblk % kXcds;
    const int64_t x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
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

// Blocks per histogram group.  A block's digit count and its exclusive
// prefix inside the group are 16-bit, so a group of G blocks of T elements
// needs (G - 1) T < 65536.
constexpr int kRsGroup = 16;
static_assert((kRsGroup - 1) * kThreads * (GS_RS_ITEMS_BIG > GS_RS_ITEMS_SMALL ? GS_RS_ITEMS_BIG : GS_RS_ITEMS_SMALL) <
                  65536, "16-bit in-group prefixes");

// ----------------------------------------------------- band row space
// A banded pass (blocks of kBandTile elements) numbers its histogram rows
// band after band: band b owns G * ceil(max(1, ceil(c_b / kBandTile)) / G)
// rows (G = kBandGroup), so no group of rows straddles two bands.  Its first
// ceil(c_b / kBandTile) rows are the blocks of its elements
// [base_b, base_b + c_b), base_b = c_0 + ... + c_{b-1}; the other rows (all
// of them for a band without pairs) count nothing.  Bases and counts are
// clipped to the capacity, as the emission drops every slot beyond it.
// Banded passes (over 2048 tiles, tens of millions of pairs) take blocks of
// 8192: half the digit bookkeeping per pair of the 4096-element block, at
// two workgroups per CU (190 VGPRs, 56 KiB of LDS); 6M Gaussians at
// 1920x1080 sort in 958 instead of 1044 us.
#ifndef GS_BAND_ITEMS
#define GS_BAND_ITEMS 32
#endif
constexpr int kBandItems = GS_BAND_ITEMS;
constexpr int kBandTile = kThreads * kBandItems;
// The banded scatter runs as 512-thread blocks of 16 pairs per thread: twice
// the wavefronts per CU of 256 threads at the same two blocks per CU (the
// 6M/1920x1080 tile sort 979 -> 893 us, 1M/1920x1080 168 -> 157 us; 1024
// threads take 1118 and 194 us).
constexpr int kBandScatterThreads = 512;
// groups of a banded pass: 8 blocks of 8192 (16 of 4096 elements)
constexpr int kBandGroup = 65536 / kBandTile;
static_assert(kBandGroup >= 1 && (kBandGroup - 1) * kBandTile < 65536, "16-bit in-group prefixes");

namespace {

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, o, 64);
        const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), o, 64);
        if (lane >= o) v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

struct BandRow {
    int64_t rows;        // rows of all bands
    int64_t row;         // logical row of this workgroup
    int band;            // its band (nb when row >= rows)
    int64_t band_base;   // first element of the band
    int64_t band_row0;   // first row of the band
    int64_t base;        // first element of the row's block
    int n_local;         // elements of the block (0: a row that counts nothing)
};

// Every wavefront computes the row space from the per-band counts (one band
// per lane) and places workgroup `wg` in it, XCD-aware like logical_block.
__device__ __forceinline__ BandRow band_row(const BandDesc& bd, int64_t wg) {
    const int lane = threadIdx.x & 63;
    const bool own = lane < bd.nb;
    const uint64_t c = own ? (uint64_t)bd.cnt[lane] : 0u;
    const uint64_t cap = (uint64_t)bd.cap;
    const uint64_t incl = wave_incl_scan64(c);
    const uint64_t base = (incl - c) < cap ? (incl - c) : cap;
    const uint64_t cl = c < cap - base ? c : cap - base;
    const uint64_t blocks = (cl + kBandTile - 1) / kBandTile;
    const uint64_t rows = own ? ((blocks > 0 ? blocks : 1) + kBandGroup - 1) / kBandGroup * kBandGroup : 0u;
    const uint64_t rend = wave_incl_scan64(rows);
    BandRow r;
    r.rows = (int64_t)shfl64(rend, 63);
    r.row = logical_block(wg, r.rows > 0 ? r.rows : 1);
    const uint64_t ended = __ballot(own && rend <= (uint64_t)r.row);
    r.band = __popcll(ended);
    r.band_base = 0;
    r.band_row0 = 0;
    r.base = 0;
    r.n_local = 0;
    if (wg >= r.rows || r.band >= bd.nb) {
        r.band = bd.nb;
        return r;
    }
    const int b = r.band;
    r.band_base = (int64_t)shfl64(base, b);
    r.band_row0 = (int64_t)(shfl64(rend, b) - shfl64(rows, b));
    const int64_t bcl = (int64_t)shfl64(cl, b);
    const int64_t i = r.row - r.band_row0;
    r.base = r.band_base + i * kBandTile;
    const int64_t left = bcl - i * kBandTile;
    r.n_local = left <= 0 ? 0 : (left < kBandTile ? (int)left : kBandTile);
    return r;
}

}  // namespace

// Histogram of 16-bit keys [first, first + count): four keys per 8-byte load
// (the order does not matter to a histogram), over the aligned quads that
// cover the range; keys of a quad outside the range are not counted.  Reads
// at most three keys on either side of the range, which the callers'
// buffers hold.
template <int BINS, int NT = kThreads>
__device__ __forceinline__ void hist16(const uint16_t* __restrict__ keys, int64_t first, int64_t count,
                                       uint32_t* h) {
    if (count <= 0) return;
    const int64_t a0 = first & ~(int64_t)3;
    const int64_t nq = (first + count - a0 + 3) >> 2;
    const int64_t last = first + count;
    constexpr int kPer = 5;   // quads per thread per round (a block's 4096 keys span at most 1025)
    for (int64_t q0 = 0; q0 < nq; q0 += (int64_t)kPer * NT) {
        uint2 v[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t q = q0 + (int64_t)k * NT + threadIdx.x;
            v[k] = q < nq ? *reinterpret_cast<const uint2*>(keys + a0 + 4 * q) : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t q = q0 + (int64_t)k * NT + threadIdx.x;
            if (q < nq) {
                const int64_t e = a0 + 4 * q;
                const uint32_t w[4] = {v[k].x & 0xFFFFu, v[k].x >> 16, v[k].y & 0xFFFFu, v[k].y >> 16};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (e + j >= first && e + j < last) atomicAdd(&h[w[j] & (uint32_t)(BINS - 1)], 1u);
            }
        }
    }
}

// KT: the key type (uint16_t keys are whole digits, shift 0).
template <int ITEMS, int BITS, typename KT, int NT = kThreads>
__global__ void __launch_bounds__(NT) k_rs_upsweep(const KT* __restrict__ keys, DevCount n, int shift,
                                                         uint16_t* __restrict__ hist) {
    constexpr int kRsTile = NT * ITEMS;
    constexpr int kRsItems = ITEMS;
    constexpr int BINS = 1 << BITS;
    __shared__ uint32_t h[BINS];
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + kRsTile - 1) / kRsTile;
    if ((int64_t)blockIdx.x >= nblk) return;
    const int64_t lb = logical_block(blockIdx.x, nblk);
    for (int d = threadIdx.x; d < BINS; d += NT) h[d] = 0u;
    __syncthreads();
    const int64_t base = lb * kRsTile;
    if constexpr (sizeof(KT) == 2) {
        hist16<BINS, NT>(keys, base, (cnt - base) < kRsTile ? (cnt - base) : kRsTile, h);
    } else {
        // (clamped, unconditional loads: a load under a per-lane condition
        // becomes a branch that waits for it)
        uint32_t k[kRsItems];
#pragma unroll
        for (int r = 0; r < kRsItems; ++r) {
            const int64_t idx = base + (int64_t)r * NT + threadIdx.x;
            k[r] = keys[idx < cnt ? idx : cnt - 1];
        }
#pragma unroll
        for (int r = 0; r < kRsItems; ++r) {
            const int64_t idx = base + (int64_t)r * NT + threadIdx.x;
            if (idx < cnt) atomicAdd(&h[(k[r] >> shift) & (uint32_t)(BINS - 1)], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < BINS; d += NT) hist[lb * BINS + d] = (uint16_t)h[d];
}

// Workgroup (g, y): digit pairs y*256 .. y*256+255 of block group g.  The
// counts of the group's blocks become their exclusive prefix inside the group
// (at most 15 x 4096, so they stay 16-bit); the group total goes to
// gsum[g][d].  A thread takes two adjacent digits, one 32-bit word of each
// 16-bit row, and loads all its words before the first store, unconditionally
// (rows past the last are clamped to it and not used).
template <int ITEMS, int BITS>
__global__ void __launch_bounds__(kThreads) k_rs_group(uint16_t* __restrict__ hist, uint32_t* __restrict__ gsum,
                                                       DevCount n) {
    constexpr int kRsTile = kThreads * ITEMS;
    constexpr int BINS = 1 << BITS;
    static_assert(BINS % 2 == 0, "digit pairs");
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + kRsTile - 1) / kRsTile;
    const int64_t g = blockIdx.x;
    const int dp = blockIdx.y * kThreads + threadIdx.x;
    if (g * kRsGroup >= nblk || 2 * dp >= BINS) return;
    uint32_t v[kRsGroup];
#pragma unroll
    for (int j = 0; j < kRsGroup; ++j) {
        const int64_t lb = g * kRsGroup + j < nblk ? g * kRsGroup + j : nblk - 1;
        v[j] = *reinterpret_cast<const uint32_t*>(hist + lb * BINS + 2 * dp);
    }
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int j = 0; j < kRsGroup; ++j) {
        const int64_t lb = g * kRsGroup + j;
        if (lb < nblk) {
            *reinterpret_cast<uint32_t*>(hist + lb * BINS + 2 * dp) = lo | (hi << 16);
            lo += v[j] & 0xFFFFu;
            hi += v[j] >> 16;
        }
    }
    *reinterpret_cast<uint2*>(gsum + g * BINS + 2 * dp) = make_uint2(lo, hi);
}

// Exclusive prefix of the group totals over the groups (in place) and the
// digit totals.  A workgroup takes 64 digits (one per lane) and splits the
// groups into 16 contiguous segments, one per wavefront.
constexpr int kGscanSegs = 16;

template <int ITEMS, int BITS>
__global__ void __launch_bounds__(64 * kGscanSegs) k_rs_gscan(uint32_t* __restrict__ gsum,
                                                              uint32_t* __restrict__ totals, DevCount n) {
    constexpr int kRsTile = kThreads * ITEMS;
    constexpr int BINS = 1 << BITS;
    __shared__ uint32_t part[kGscanSegs][64];
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + kRsTile - 1) / kRsTile;
    const int64_t ngrp = (nblk + kRsGroup - 1) / kRsGroup;
    const int dl = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int d = blockIdx.x * 64 + dl;
    const bool own = d < BINS;
    const int64_t len = (ngrp + kGscanSegs - 1) / kGscanSegs;
    const int64_t g0 = seg * len;
    const int64_t g1 = (g0 + len < ngrp) ? g0 + len : ngrp;
    uint32_t sum = 0;
    if (own) {
#pragma unroll 8
        for (int64_t g = g0; g < g1; ++g) sum += gsum[g * BINS + d];
    }
    part[seg][dl] = sum;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kGscanSegs; ++k) {
        const uint32_t v = part[k][dl];
        pre += k < seg ? v : 0u;
        tot += v;
    }
    if (own) {
        // in chunks of 8 groups, loads before stores
        uint32_t run = pre;
        for (int64_t c0 = g0; c0 < g1; c0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = c0 + k < g1 ? gsum[(c0 + k) * BINS + d] : 0u;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (c0 + k < g1) gsum[(c0 + k) * BINS + d] = run;
                run += v[k];
            }
        }
        if (seg == 0) totals[d] = tot;
    }
}

// Steps 2 and 3 in one launch, for passes with few groups: a workgroup takes
// 64 digits (one per lane) and 16 contiguous segments of the groups (one per
// wavefront); each lane makes its groups' in-group prefixes and totals, then
// the segments' totals are scanned in LDS and the group totals turned into
// their exclusive prefix.
template <int ITEMS, int BITS>
__global__ void __launch_bounds__(64 * kGscanSegs) k_rs_groupscan(uint16_t* __restrict__ hist,
                                                                  uint32_t* __restrict__ gsum,
                                                                  uint32_t* __restrict__ totals, DevCount n) {
    constexpr int kRsTile = kThreads * ITEMS;
    constexpr int BINS = 1 << BITS;
    __shared__ uint32_t part[kGscanSegs][64];
    const int64_t cnt = dev_count(n);
    const int64_t nblk = (cnt + kRsTile - 1) / kRsTile;
    const int64_t ngrp = (nblk + kRsGroup - 1) / kRsGroup;
    const int dl = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int d = blockIdx.x * 64 + dl;
    const bool own = d < BINS;
    const int64_t len = (ngrp + kGscanSegs - 1) / kGscanSegs;
    const int64_t g0 = seg * len;
    const int64_t g1 = (g0 + len < ngrp) ? g0 + len : ngrp;
    uint32_t sum = 0;
    if (own) {
        for (int64_t g = g0; g < g1; ++g) {
            uint32_t v[kRsGroup];
#pragma unroll
            for (int j = 0; j < kRsGroup; ++j) {
                const int64_t lb = g * kRsGroup + j;
                v[j] = lb < nblk ? hist[lb * BINS + d] : 0u;
            }
            uint32_t run = 0;
#pragma unroll
            for (int j = 0; j < kRsGroup; ++j) {
                const int64_t lb = g * kRsGroup + j;
                if (lb < nblk) hist[lb * BINS + d] = (uint16_t)run;
                run += v[j];
            }
            gsum[g * BINS + d] = run;
            sum += run;
        }
    }
    part[seg][dl] = sum;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kGscanSegs; ++k) {
        const uint32_t v = part[k][dl];
        pre += k < seg ? v : 0u;
        tot += v;
    }
    if (own) {
        // in chunks of 8 groups, loads before stores
        uint32_t run = pre;
        for (int64_t c0 = g0; c0 < g1; c0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = c0 + k < g1 ? gsum[(c0 + k) * BINS + d] : 0u;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (c0 + k < g1) gsum[(c0 + k) * BINS + d] = run;
                run += v[k];
            }
        }
        if (seg == 0) totals[d] = tot;
    }
}

// N consecutive 32-bit (load_run) or 16-bit (load_run16) words from an
// address aligned to their total size, in as few vector loads as possible.
template <int N>
__device__ __forceinline__ void load_run(const uint32_t* __restrict__ p, uint32_t* v) {
    if constexpr (N % 4 == 0) {
#pragma unroll
        for (int k = 0; k < N / 4; ++k) {
            const uint4 q = reinterpret_cast<const uint4*>(p)[k];
            v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
        }
    } else if constexpr (N == 2) {
        const uint2 q = *reinterpret_cast<const uint2*>(p);
        v[0] = q.x; v[1] = q.y;
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = p[k];
    }
}

template <int N>
__device__ __forceinline__ void load_run16(const uint16_t* __restrict__ p, uint32_t* v) {
    if constexpr (N % 8 == 0) {
#pragma unroll
        for (int k = 0; k < N / 8; ++k) {
            const uint4 q = reinterpret_cast<const uint4*>(p)[k];
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) { v[8 * k + 2 * j] = w[j] & 0xFFFFu; v[8 * k + 2 * j + 1] = w[j] >> 16; }
        }
    } else if constexpr (N == 4) {
        const uint2 q = *reinterpret_cast<const uint2*>(p);
        v[0] = q.x & 0xFFFFu; v[1] = q.x >> 16; v[2] = q.y & 0xFFFFu; v[3] = q.y >> 16;
    } else if constexpr (N == 2) {
        const uint32_t q = *reinterpret_cast<const uint32_t*>(p);
        v[0] = q & 0xFFFFu; v[1] = q >> 16;
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = p[k];
    }
}

// Stable scatter of one pass.  The digit start offsets are the exclusive scan
// of the digit totals, recomputed by every block instead of by another launch.
// ranges != nullptr: the digit is the whole tile id, and the first workgroup
// also writes ranges[t] = [start, start + total) (or [0, 0) when empty) for
// t < n_ranges; it does so even when there is nothing to sort.
// LDS of one scatter block, 32-bit words: the per-wavefront digit counters
// (phases 1-3), followed by the digit scans' kWaves + 1 words (phase 2),
// share their words with the block's reordered elements (phases 3-4): keys
// (or 16-bit digits), values and second values.  (Sharing the scan words
// keeps the tile sort's block at 32 KiB with its digit offsets: five blocks
// per CU.)
template <int ITEMS, bool V2, bool KEYS, int BITS, int NT = kThreads>
struct ScatterLds {
    static constexpr int kWaves = NT / 64;
    static constexpr int kTile = NT * ITEMS;
    static constexpr int kHalf = (1 << BITS) >= 2 ? (1 << BITS) / 2 : 1;
    static constexpr int kCounters = kWaves * kHalf;
    static constexpr int kScan = kCounters;   // first word of the scan words
    static constexpr int kKeyWords = KEYS ? kTile : kTile / 2;
    static constexpr int kData = kKeyWords + kTile + (V2 ? kTile : 0);
    static constexpr int kWords = kCounters + kWaves + 1 > kData ? kCounters + kWaves + 1 : kData;
};

// BAND: a banded pass (see band_row); keys are band-local tile ids, every
// band's first row writes the band's tile ranges, and positions are offset
// by the band's first element.
template <int ITEMS, bool V2, bool KEYS, int BITS, bool BAND, typename KT, int NT = kThreads>
// At least four waves per SIMD: the registers let the compiler issue the
// element loads and the digit bookkeeping's loads back to back, ahead of the
// ranking (at five it serialised the latter, each load waiting for the last,
// in the 256-thread form of 16 elements per thread).
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_rs_downsweep(const KT* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           const uint32_t* __restrict__ vals2_in,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out,
                                                           uint32_t* __restrict__ vals2_out, DevCount n, int shift,
                                                           const uint16_t* __restrict__ hist,
                                                           const uint32_t* __restrict__ gsum,
                                                           const uint32_t* __restrict__ totals,
                                                           uint32_t* __restrict__ ranges, int64_t n_ranges,
                                                           BandDesc bd) {
    constexpr int kRsTile = NT * ITEMS;
    constexpr int NW = NT / 64;
    static_assert(!BAND || ITEMS * NT == kBandTile, "banded passes use blocks of kBandTile");
    static_assert(sizeof(KT) == 4 || !KEYS, "16-bit keys are not written out");
    constexpr int kRsItems = ITEMS;
    constexpr int BINS = 1 << BITS;
    constexpr uint32_t MASK = (uint32_t)BINS - 1u;
    constexpr int DPT = BINS >= NT ? BINS / NT : 1;   // digits per thread in the digit scans
    constexpr int HALF = BINS >= 2 ? BINS / 2 : 1;
    // per wavefront and digit a 16-bit count (two digits per word): first the
    // running count, then the wavefront's start position in the block; once
    // every element has its position, the same words hold the block in digit
    // order: keys when they are written out, else only the digits (16-bit),
    // then the values (and second values)
    using Lds = ScatterLds<ITEMS, V2, KEYS, BITS, NT>;
    __shared__ uint32_t lds[Lds::kWords];
    uint32_t (*wcnt)[HALF] = reinterpret_cast<uint32_t(*)[HALF]>(lds);
    uint32_t* skey = lds;
    uint16_t* sdig = reinterpret_cast<uint16_t*>(lds);
    uint32_t* sval = lds + Lds::kKeyWords;
    uint32_t* sval2 = lds + Lds::kKeyWords + kRsTile;
    __shared__ int32_t gofs[BINS];
    uint32_t* scratch = lds + Lds::kScan;
    int64_t cnt, lb, base, band_base = 0;
    int n_local, band = 0;
    bool active, do_ranges;
    if constexpr (BAND) {
        const BandRow br = band_row(bd, blockIdx.x);
        if (br.band >= bd.nb) return;
        cnt = bd.cap;
        lb = br.row;
        base = br.base;
        n_local = br.n_local;
        band = br.band;
        band_base = br.band_base;
        active = n_local > 0;
        do_ranges = lb == br.band_row0;
    } else {
        cnt = dev_count(n);
        const int64_t nblk = (cnt + kRsTile - 1) / kRsTile;
        active = (int64_t)blockIdx.x < nblk;
        do_ranges = ranges != nullptr && blockIdx.x == 0;
        lb = active ? logical_block(blockIdx.x, nblk) : 0;
        base = lb * kRsTile;
        n_local = active ? (int)((cnt - base) < kRsTile ? (cnt - base) : kRsTile) : 0;
    }
    if (!active && !do_ranges) return;
    const int64_t grp = lb / (BAND ? kBandGroup : kRsGroup);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t* __restrict__ dtot = BAND ? totals + (int64_t)band * BINS : totals;
    const int64_t rlimit = BAND ? (int64_t)bd.ntiles[band] : n_ranges;
    uint32_t* __restrict__ rout = BAND ? ranges + 2 * (int64_t)bd.tile0[band] : ranges;

    for (int e = threadIdx.x; e < NW * HALF; e += NT) (&wcnt[0][0])[e] = 0u;
    __syncthreads();

    // phase 1: keys in registers; per element its position among the
    // elements of its wavefront holding the same digit.  Every lane loads
    // (lanes past the block's end reload its last element, and a workgroup
    // without elements its first): a load under a per-lane condition becomes
    // a branch, at whose end the compiler waits for it, so the rows' loads
    // would not overlap.
    const int wbase = wave * 64 * kRsItems;
    const int last = n_local > 0 ? n_local - 1 : 0;
    const int64_t lbase = n_local > 0 ? base : 0;   // (element 0 exists whenever a pass is launched)
    // (the values are loaded only when they are placed, in phase 3, so they
    // take no registers through the ranking and the digit scans)
    uint32_t key[kRsItems], info[kRsItems];
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int li = wbase + r * 64 + lane;
        key[r] = keys_in[lbase + (li < last ? li : last)];
    }
    // the digit bookkeeping's global reads (a few vector loads per thread),
    // issued before the ranking so that their latency overlaps it
    // (unconditional loads, as above: a digit past the last, or a row of a
    // workgroup without elements, reads a valid word and is masked after)
    const int d0 = threadIdx.x * DPT;
    const bool owner = d0 < BINS;
    const int dl = owner ? d0 : 0;   // a thread without digits reads digit 0's words
    uint32_t tg[DPT], hb[DPT];
    load_run<DPT>(dtot + dl, tg);
    {
        uint32_t gs[DPT], hs[DPT];
        load_run<DPT>(gsum + grp * BINS + dl, gs);
        load_run16<DPT>(hist + lb * BINS + dl, hs);
#pragma unroll
        for (int k = 0; k < DPT; ++k) hb[k] = (owner && active) ? gs[k] + hs[k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < DPT; ++k) tg[k] = owner ? tg[k] : 0u;
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int li = wbase + r * 64 + lane;
        const uint32_t d = (key[r] >> shift) & MASK;
        // the wavefront's count of digit d so far: the LDS applies the
        // same-address adds of one instruction in lane order, and the rows'
        // instructions in issue order, so the returned count is this
        // element's rank among the wavefront's earlier elements of digit d
        // (the digit is kept beside it, bits 16 up, so the key need not stay
        // live when it is not written out).  The add stays under the lane's
        // condition: unconditional adds (lanes without an element on a spare
        // word) let the compiler keep every row's operands live at once and
        // spill.
        info[r] = d << 16;
        if (li < n_local) {
            const uint32_t old = atomicAdd(&wcnt[wave][d >> 1], 1u << (16 * (d & 1u)));
            info[r] |= (old >> (16 * (d & 1u))) & 0xFFFFu;
        }
    }
    __syncthreads();

    // phase 2: digit starts (global and block-local), per-wave start positions
    {
        uint32_t gtot = 0, lsum = 0;
#pragma unroll
        for (int k = 0; k < DPT; ++k) gtot += tg[k];
        // DPT >= 2: the thread's digits come in pairs sharing a counter word,
        // and sums of such words are sums of both halves (no half exceeds
        // 4096).  A thread rewrites only its own words, so it reads them
        // again after the scans instead of keeping them in registers.
        constexpr int NP = DPT >= 2 ? DPT / 2 : 1;
        uint32_t cw1[NW];   // DPT == 1: this thread's halves
        if constexpr (DPT >= 2) {
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                uint32_t sw = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) sw += owner ? wcnt[w][(d0 >> 1) + q] : 0u;
                lsum += (sw & 0xFFFFu) + (sw >> 16);
            }
        } else {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                cw1[w] = owner ? (wcnt[w][d0 >> 1] >> (16 * (d0 & 1))) & 0xFFFFu : 0u;
                lsum += cw1[w];
            }
        }
        uint32_t all;
        uint32_t grun = block_excl_scan<NW>(gtot, scratch, all);
        uint32_t lrun = block_excl_scan<NW>(lsum, scratch, all);
        if (owner) {
            // digit d of this thread: its offset (global start of the digit,
            // plus the digit's count in the blocks before, minus its start in
            // this block), and the tile range when the digit is a tile
            auto digit = [&](int k, uint32_t tl) {
                const int d = d0 + k;
                // positions stay below the capacity (at most 2^31)
                gofs[d] = (int32_t)((uint32_t)band_base + grun + hb[k]) - (int32_t)lrun;
                if (do_ranges && d < rlimit) {
                    const uint32_t s0 = (uint32_t)band_base + grun;
                    const uint2 rg = tg[k] ? make_uint2(s0, s0 + tg[k]) : make_uint2(0u, 0u);
                    reinterpret_cast<uint2*>(rout)[d] = rg;
                }
                grun += tg[k];
                lrun += tl;
            };
            if constexpr (DPT >= 2) {
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    uint32_t c[NW], sw = 0;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        c[w] = wcnt[w][(d0 >> 1) + q];
                        sw += c[w];
                    }
                    const uint32_t st0 = lrun;
                    digit(2 * q, sw & 0xFFFFu);
                    const uint32_t st1 = lrun;
                    digit(2 * q + 1, sw >> 16);
                    uint32_t run = st0 | (st1 << 16);
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        wcnt[w][(d0 >> 1) + q] = run;
                        run += c[w];
                    }
                }
            } else {
                // one digit per thread: the two halves of a word belong to two threads
                uint32_t run = lrun;
                digit(0, lsum);
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    reinterpret_cast<uint16_t*>(&wcnt[w][0])[d0] = (uint16_t)run;
                    run += cw1[w];
                }
            }
        }
    }
    __syncthreads();

    // phase 3: stable local placement in LDS; every position is read from the
    // counters before the (aliased) element words are written
    uint32_t val[kRsItems], val2[V2 ? kRsItems : 1];
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int li = wbase + r * 64 + lane;
        const int64_t e = lbase + (li < last ? li : last);
        val[r] = vals_in ? vals_in[e] : (uint32_t)e;
        // the second value travels with the element, read at its position
        // (a coalesced read, where a gather by the value would fetch a
        // cache line per element once the array outgrows the L2)
        if (V2) val2[V2 ? r : 0] = vals2_in[e];
    }
    uint32_t pos[kRsItems];
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int li = wbase + r * 64 + lane;
        const uint32_t d = info[r] >> 16;
        const uint32_t start = (wcnt[wave][d >> 1] >> (16 * (d & 1u))) & 0xFFFFu;
        pos[r] = li < n_local ? start + (info[r] & 0xFFFFu) : 0xFFFFFFFFu;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        if (pos[r] < (uint32_t)kRsTile) {
            if (KEYS)
                skey[pos[r]] = key[r];
            else
                sdig[pos[r]] = (uint16_t)(info[r] >> 16);
            sval[pos[r]] = val[r];
            if (V2) sval2[pos[r]] = val2[V2 ? r : 0];
        }
    }
    __syncthreads();

    // phase 4: coalesced write-out, digit runs are contiguous in LDS and in memory
    for (int i = threadIdx.x; i < n_local; i += NT) {
        const uint32_t k = KEYS ? skey[i] : 0u;
        const uint32_t d = KEYS ? (k >> shift) & MASK : (uint32_t)sdig[i];
        const int64_t gpos = (int64_t)gofs[d] + i;
        if (gpos >= 0 && gpos < cnt) {
            vals_out[gpos] = sval[i];
            if (V2) vals2_out[gpos] = sval2[i];
            if (KEYS) keys_out[gpos] = k;
        }
    }
}

static int rs_tile(int64_t cap) { return kThreads * (cap >= kBigPass ? kRsItemsBig : kRsItemsSmall); }

int64_t rs_pass_blocks(int64_t cap) { return (cap + rs_tile(cap) - 1) / rs_tile(cap); }

int64_t rs_hist_bytes(int64_t cap) {
    const int64_t nb = rs_pass_blocks(cap) > 0 ? rs_pass_blocks(cap) : 1;
    const int64_t ng = (nb + kRsGroup - 1) / kRsGroup;
    // 16-bit block rows, then (256-byte aligned) 32-bit group rows
    return ((nb * kRsMaxBins * 2 + 255) / 256) * 256 + ng * kRsMaxBins * 4;
}

// Block widths of the scatter (the histogram passes keep 256 threads, except
// for the small 32-bit passes), all on the same partition into blocks of
// 256 x ITEMS elements:
//  - 32-bit keys, fewer than 4M (a frame's depth sort: one block per CU or
//    fewer): histogram and scatter as 1024-thread blocks, more wavefronts per
//    CU to hide the loads' and the ranking's latency where the grid gives
//    each SIMD only one (1M depth keys: 77.8 -> 73.0 us; 512 threads measured
//    alike, 2048-key blocks slower);
//  - every other pass: 512-thread scatter blocks, twice the wavefronts of
//    256 threads at the same blocks per CU (6M depth keys 233 -> 218 us, the
//    tile sort of 10.8M pairs at 960x540 66.1 -> 65.4 us and of 64.7M pairs
//    375 -> 355 us; 1024 threads are slower there: 75 us at 10.8M pairs).
constexpr int kSmallPassThreads = 1024;
constexpr int kScatterThreads = 512;

template <int ITEMS, bool V2, int BITS, typename KT, int NT>
static void launch_scatter(const KT* keys_in, const uint32_t* vals_in, const uint32_t* vals2_in, uint32_t* keys_out,
                           uint32_t* vals_out, uint32_t* vals2_out, DevCount n, int shift, const uint16_t* hist,
                           const uint32_t* gsum, uint32_t* totals, uint32_t* ranges, int64_t n_ranges, int64_t nblk,
                           hipStream_t st) {
    const BandDesc none{};
    if constexpr (sizeof(KT) == 4) {
        if (keys_out) {
            hipLaunchKernelGGL((k_rs_downsweep<ITEMS, V2, true, BITS, false, KT, NT>), dim3((unsigned)nblk), dim3(NT),
                               0, st, keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift, hist, gsum,
                               totals, ranges, n_ranges, none);
            return;
        }
    }
    hipLaunchKernelGGL((k_rs_downsweep<ITEMS, V2, false, BITS, false, KT, NT>), dim3((unsigned)nblk), dim3(NT), 0, st,
                       keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift, hist, gsum, totals, ranges,
                       n_ranges, none);
}

template <int ITEMS, bool V2, int BITS, typename KT>
static void launch_pass(const KT* keys_in, const uint32_t* vals_in, const uint32_t* vals2_in,
                        uint32_t* keys_out, uint32_t* vals_out, uint32_t* vals2_out, DevCount n, int shift,
                        void* hist_scratch, uint32_t* totals, uint32_t* ranges, int64_t n_ranges, hipStream_t st) {
    constexpr int BINS = 1 << BITS;
    const int64_t nb = rs_pass_blocks(n.cap);
    const int64_t nblk = nb > 0 ? nb : 1;
    const int64_t ngrp = (nblk + kRsGroup - 1) / kRsGroup;
    uint16_t* hist = static_cast<uint16_t*>(hist_scratch);
    uint32_t* gsum = reinterpret_cast<uint32_t*>(static_cast<char*>(hist_scratch) +
                                                 ((nblk * kRsMaxBins * 2 + 255) / 256) * 256);
    const unsigned dgrid = (unsigned)((BINS / 2 + kThreads - 1) / kThreads);   // digit pairs (k_rs_group)
    constexpr int kWideItems = ITEMS * kThreads / kSmallPassThreads;
    static_assert(kWideItems * kSmallPassThreads == ITEMS * kThreads, "same block partition");
    constexpr bool k32 = sizeof(KT) == 4;
    const bool wide = k32 && n.cap < kBigPass;
    if constexpr (k32) {
        if (wide)
            hipLaunchKernelGGL((k_rs_upsweep<kWideItems, BITS, KT, kSmallPassThreads>), dim3((unsigned)nblk),
                               dim3(kSmallPassThreads), 0, st, keys_in, n, shift, hist);
    }
    if constexpr (!k32) {
        // 16-bit tile ids: the histogram as 512-thread blocks too (the tile
        // sort of 10.8M pairs at 960x540 65.6 -> 63.8 us; the banded pass's
        // histogram measured slower that way and keeps 256)
        hipLaunchKernelGGL((k_rs_upsweep<ITEMS * kThreads / kScatterThreads, BITS, KT, kScatterThreads>),
                           dim3((unsigned)nblk), dim3(kScatterThreads), 0, st, keys_in, n, shift, hist);
    } else if (!wide) {
        hipLaunchKernelGGL((k_rs_upsweep<ITEMS, BITS, KT>), dim3((unsigned)nblk), dim3(kThreads), 0, st, keys_in, n,
                           shift, hist);
    }
    if (n.cap < kBigPass) {
        hipLaunchKernelGGL((k_rs_groupscan<ITEMS, BITS>), dim3((unsigned)((BINS + 63) / 64)), dim3(64 * kGscanSegs), 0,
                           st, hist, gsum, totals, n);
    } else {
        hipLaunchKernelGGL((k_rs_group<ITEMS, BITS>), dim3((unsigned)ngrp, dgrid), dim3(kThreads), 0, st, hist, gsum,
                           n);
        hipLaunchKernelGGL((k_rs_gscan<ITEMS, BITS>), dim3((unsigned)((BINS + 63) / 64)), dim3(64 * kGscanSegs), 0,
                           st, gsum, totals, n);
    }
    if constexpr (k32) {
        if (wide) {
            launch_scatter<kWideItems, V2, BITS, KT, kSmallPassThreads>(keys_in, vals_in, vals2_in, keys_out, vals_out,
                                                                        vals2_out, n, shift, hist, gsum, totals,
                                                                        ranges, n_ranges, nblk, st);
            return;
        }
    }
    static_assert(ITEMS * kThreads % kScatterThreads == 0, "same block partition");
    launch_scatter<ITEMS * kThreads / kScatterThreads, V2, BITS, KT, kScatterThreads>(
        keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift, hist, gsum, totals, ranges, n_ranges, nblk,
        st);
}

template <bool V2, typename KT>
static hipError_t dispatch_pass(int bits, const KT* keys_in, const uint32_t* vals_in,
                                const uint32_t* vals2_in, uint32_t* keys_out, uint32_t* vals_out,
                                uint32_t* vals2_out, DevCount n, int shift, void* hist, uint32_t* totals,
                                uint32_t* ranges, int64_t n_ranges, hipStream_t st) {
#define GS_RS_CASE(B)                                                                                       \
    case B:                                                                                                 \
        if (n.cap >= kBigPass)                                                                              \
            launch_pass<kRsItemsBig, V2, B, KT>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, \
                                            shift, hist, totals, ranges, n_ranges, st);                     \
        else                                                                                                \
            launch_pass<kRsItemsSmall, V2, B, KT>(keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out,  \
                                                  n, shift, hist, totals, ranges, n_ranges, st);            \
        break;
    switch (bits) {
        GS_RS_CASE(1) GS_RS_CASE(2) GS_RS_CASE(3) GS_RS_CASE(4) GS_RS_CASE(5) GS_RS_CASE(6)
        GS_RS_CASE(7) GS_RS_CASE(8) GS_RS_CASE(9) GS_RS_CASE(10) GS_RS_CASE(11)
        default: return hipErrorInvalidValue;
    }
#undef GS_RS_CASE
    return hipGetLastError();
}

hipError_t radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, const uint32_t* vals2_in,
                      uint32_t* keys_out, uint32_t* vals_out, uint32_t* vals2_out, DevCount n, int shift, int bits,
                      void* hist, uint32_t* totals, uint32_t* ranges, int64_t n_ranges, hipStream_t st) {
    if (bits < 1 || bits > kRsMaxBits) return hipErrorInvalidValue;
    if ((vals2_in == nullptr) != (vals2_out == nullptr)) return hipErrorInvalidValue;
    if (ranges != nullptr && (n_ranges < 0 || n_ranges > ((int64_t)1 << bits) || shift != 0))
        return hipErrorInvalidValue;
    if (n.cap == 0) return ranges ? launch_fill_u32(ranges, 0u, 2 * n_ranges, st) : hipSuccess;
    if (vals2_in)
        return dispatch_pass<true, uint32_t>(bits, keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift,
                                             hist, totals, ranges, n_ranges, st);
    return dispatch_pass<false, uint32_t>(bits, keys_in, vals_in, vals2_in, keys_out, vals_out, vals2_out, n, shift,
                                          hist, totals, ranges, n_ranges, st);
}

hipError_t radix_pass_tiles(const uint16_t* keys_in, const uint32_t* vals_in, uint32_t* vals_out, DevCount n,
                            int bits, void* hist, uint32_t* totals, uint32_t* ranges, int64_t n_ranges,
                            hipStream_t st) {
    if (bits < 1 || bits > kRsMaxBits || !vals_in || !ranges) return hipErrorInvalidValue;
    if (n_ranges < 0 || n_ranges > ((int64_t)1 << bits)) return hipErrorInvalidValue;
    if (n.cap == 0) return launch_fill_u32(ranges, 0u, 2 * n_ranges, st);
    return dispatch_pass<false, uint16_t>(bits, keys_in, vals_in, nullptr, nullptr, vals_out, nullptr, n, 0, hist,
                                          totals, ranges, n_ranges, st);
}

// ------------------------------------------------------------ banded tile sort

// Histogram row of every row of the band row space (zeros for rows that
// count nothing).
template <int BITS>
__global__ void __launch_bounds__(kThreads) k_band_upsweep(const uint16_t* __restrict__ keys, BandDesc bd,
                                                           uint16_t* __restrict__ hist) {
    constexpr int BINS = 1 << BITS;
    __shared__ uint32_t h[BINS];
    const BandRow br = band_row(bd, blockIdx.x);
    if (br.band >= bd.nb) return;
    for (int d = threadIdx.x; d < BINS; d += kThreads) h[d] = 0u;
    __syncthreads();
    hist16<BINS>(keys, br.base, br.n_local, h);
    __syncthreads();
    for (int d = threadIdx.x; d < BINS; d += kThreads) hist[br.row * BINS + d] = (uint16_t)h[d];
}

// In-group prefixes of the rows' counts and the group totals, over the
// groups of the whole row space (no group straddles two bands; every group
// is whole), two adjacent digits per thread as in k_rs_group.
template <int BITS>
__global__ void __launch_bounds__(kThreads) k_band_group(uint16_t* __restrict__ hist, uint32_t* __restrict__ gsum,
                                                         BandDesc bd) {
    constexpr int BINS = 1 << BITS;
    static_assert(BINS % 2 == 0, "digit pairs");
    const BandRow br = band_row(bd, 0);
    const int64_t g = blockIdx.x;
    const int dp = blockIdx.y * kThreads + threadIdx.x;
    if (g * kBandGroup >= br.rows || 2 * dp >= BINS) return;
    uint32_t v[kBandGroup];
#pragma unroll
    for (int j = 0; j < kBandGroup; ++j)
        v[j] = *reinterpret_cast<const uint32_t*>(hist + (g * kBandGroup + j) * BINS + 2 * dp);
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int j = 0; j < kBandGroup; ++j) {
        *reinterpret_cast<uint32_t*>(hist + (g * kBandGroup + j) * BINS + 2 * dp) = lo | (hi << 16);
        lo += v[j] & 0xFFFFu;
        hi += v[j] >> 16;
    }
    *reinterpret_cast<uint2*>(gsum + g * BINS + 2 * dp) = make_uint2(lo, hi);
}

// Workgroup (x, b): digits 64 x .. 64 x + 63 of band b.  The group totals of
// the band's groups become their exclusive prefix inside the band, and the
// band's digit totals go to totals[b][d].
template <int BITS>
__global__ void __launch_bounds__(64 * kGscanSegs) k_band_gscan(uint32_t* __restrict__ gsum,
                                                                uint32_t* __restrict__ totals, BandDesc bd) {
    constexpr int BINS = 1 << BITS;
    __shared__ uint32_t part[kGscanSegs][64];
    const int b = blockIdx.y;
    // the band's rows: the row space placement of its first row
    const int lane_b = threadIdx.x & 63;
    const bool own = lane_b < bd.nb;
    const uint64_t c = own ? (uint64_t)bd.cnt[lane_b] : 0u;
    const uint64_t cap = (uint64_t)bd.cap;
    const uint64_t incl = wave_incl_scan64(c);
    const uint64_t base = (incl - c) < cap ? (incl - c) : cap;
    const uint64_t cl = c < cap - base ? c : cap - base;
    const uint64_t blocks = (cl + kBandTile - 1) / kBandTile;
    const uint64_t rows = own ? ((blocks > 0 ? blocks : 1) + kBandGroup - 1) / kBandGroup * kBandGroup : 0u;
    const uint64_t rend = wave_incl_scan64(rows);
    const int64_t gb = (int64_t)((shfl64(rend, b) - shfl64(rows, b)) / kBandGroup);
    const int64_t ge = (int64_t)(shfl64(rend, b) / kBandGroup);
    const int dl = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int d = blockIdx.x * 64 + dl;
    const bool mine = d < BINS;
    const int64_t len = (ge - gb + kGscanSegs - 1) / kGscanSegs;
    const int64_t g0 = gb + seg * len < ge ? gb + seg * len : ge;
    const int64_t g1 = (g0 + len < ge) ? g0 + len : ge;
    uint32_t sum = 0;
    if (mine) {
        // in chunks of 8 groups, every load issued before the sums
        for (int64_t c0 = g0; c0 < g1; c0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = gsum[(c0 + k < g1 ? c0 + k : g1 - 1) * BINS + d];
#pragma unroll
            for (int k = 0; k < 8; ++k) sum += c0 + k < g1 ? v[k] : 0u;
        }
    }
    part[seg][dl] = sum;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kGscanSegs; ++k) {
        const uint32_t v = part[k][dl];
        pre += k < seg ? v : 0u;
        tot += v;
    }
    if (mine) {
        uint32_t run = pre;
        for (int64_t c0 = g0; c0 < g1; c0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = c0 + k < g1 ? gsum[(c0 + k) * BINS + d] : 0u;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (c0 + k < g1) gsum[(c0 + k) * BINS + d] = run;
                run += v[k];
            }
        }
        if (seg == 0) totals[(int64_t)b * BINS + d] = tot;
    }
}

static int64_t band_rows_max(int64_t cap, int nb) {
    return (cap + kBandTile - 1) / kBandTile + (int64_t)kBandGroup * nb;
}

int64_t seg_hist_bytes(int64_t cap, int nb) {
    const int64_t rows = band_rows_max(cap, nb);
    return ((rows * kRsMaxBins * 2 + 255) / 256) * 256 + (rows / kBandGroup + 1) * kRsMaxBins * 4;
}

template <int BITS>
static void launch_band_pass(const uint16_t* keys_in, const uint32_t* vals_in, uint32_t* vals_out,
                             const BandDesc& bd, void* hist_scratch, uint32_t* totals, uint32_t* ranges,
                             hipStream_t st) {
    constexpr int BINS = 1 << BITS;
    const int64_t rows = band_rows_max(bd.cap, bd.nb);
    uint16_t* hist = static_cast<uint16_t*>(hist_scratch);
    uint32_t* gsum = reinterpret_cast<uint32_t*>(static_cast<char*>(hist_scratch) +
                                                 ((rows * kRsMaxBins * 2 + 255) / 256) * 256);
    const unsigned dgrid = (unsigned)((BINS / 2 + kThreads - 1) / kThreads);   // digit pairs
    hipLaunchKernelGGL((k_band_upsweep<BITS>), dim3((unsigned)rows), dim3(kThreads), 0, st, keys_in, bd, hist);
    hipLaunchKernelGGL((k_band_group<BITS>), dim3((unsigned)(rows / kBandGroup), dgrid), dim3(kThreads), 0, st, hist,
                       gsum, bd);
    hipLaunchKernelGGL((k_band_gscan<BITS>), dim3((unsigned)((BINS + 63) / 64), (unsigned)bd.nb),
                       dim3(64 * kGscanSegs), 0, st, gsum, totals, bd);
    const DevCount unused{nullptr, bd.cap};
    hipLaunchKernelGGL((k_rs_downsweep<kBandTile / kBandScatterThreads, false, false, BITS, true, uint16_t,
                                       kBandScatterThreads>),
                       dim3((unsigned)rows), dim3(kBandScatterThreads), 0, st, keys_in, vals_in, nullptr, nullptr,
                       vals_out, nullptr, unused, 0, hist, gsum, totals, ranges, (int64_t)0, bd);
}

hipError_t radix_pass_banded(const uint16_t* keys_in, const uint32_t* vals_in, uint32_t* vals_out,
                             const BandDesc& bands, int bits, void* hist, uint32_t* totals, uint32_t* ranges,
                             hipStream_t st) {
    if (bits < 1 || bits > kRsMaxBits || bands.nb < 1 || bands.nb > kMaxBands || !ranges || !vals_in)
        return hipErrorInvalidValue;
    for (int b = 0; b < bands.nb; ++b)
        if (bands.ntiles[b] > (1u << bits)) return hipErrorInvalidValue;
#define GS_BAND_CASE(B)                                                                \
    case B:                                                                            \
        launch_band_pass<B>(keys_in, vals_in, vals_out, bands, hist, totals, ranges, st); \
        break;
    switch (bits) {
        GS_BAND_CASE(1) GS_BAND_CASE(2) GS_BAND_CASE(3) GS_BAND_CASE(4) GS_BAND_CASE(5) GS_BAND_CASE(6)
        GS_BAND_CASE(7) GS_BAND_CASE(8) GS_BAND_CASE(9) GS_BAND_CASE(10) GS_BAND_CASE(11)
        default: return hipErrorInvalidValue;
    }
#undef GS_BAND_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------------ pair counts

// Tile counts of depth-order chunks: part[c] over positions [256 c, 256 c + 256)
// and sup[s] over [4096 s, 4096 s + 4096); the grand total (the pair count)
// is added to *total, which the caller has zeroed.  The emission derives each
// block's first slot from these counts.
template <bool kGather>
__global__ void __launch_bounds__(kThreads) k_chunk_counts(const uint32_t* __restrict__ rects,
                                                           const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ touched, int64_t n,
                                                           uint32_t* __restrict__ part, uint32_t* __restrict__ sup,
                                                           uint32_t* __restrict__ total) {
    __shared__ uint32_t wsum[kWaves];
    constexpr int kPer = kSuperChunk / kThreads;   // 16 consecutive positions per thread
    const int64_t first = (int64_t)blockIdx.x * kSuperChunk + (int64_t)threadIdx.x * kPer;
    uint32_t sum = 0;
    if (kGather) {
        // the projection's counts, through the depth order (culled Gaussians count 0)
        uint32_t gi[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) gi[k] = first + k < n ? order[first + k] : 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < kPer; ++k) sum += (int64_t)gi[k] < n ? touched[gi[k]] : 0u;
    } else {
        // all four 16-byte loads first (a thread past the end reloads the
        // first quad and counts nothing), then the arithmetic: left to
        // itself the scheduler interleaves each load with its use, so they
        // do not overlap
        const bool whole = first + kPer <= n;
        const uint4* r4 = reinterpret_cast<const uint4*>(rects + (whole ? first : 0));
        uint4 q[kPer / 4];
#pragma unroll
        for (int k = 0; k < kPer / 4; ++k) q[k] = r4[k];
        __builtin_amdgcn_sched_barrier(0);
        if (whole) {
#pragma unroll
            for (int k = 0; k < kPer / 4; ++k)
                sum += rect_tiles(q[k].x) + rect_tiles(q[k].y) + rect_tiles(q[k].z) + rect_tiles(q[k].w);
        } else {
            for (int k = 0; k < kPer; ++k)
                if (first + k < n) sum += rect_tiles(rects[first + k]);
        }
    }
    // 16 consecutive threads cover one 256-position chunk
    uint32_t c = sum;
#pragma unroll
    for (int o = 1; o < kChunk / kPer; o <<= 1) c += (uint32_t)__shfl_xor((int)c, o, 64);
    const int64_t ci = (int64_t)blockIdx.x * (kSuperChunk / kChunk) + threadIdx.x / (kChunk / kPer);
    if ((threadIdx.x % (kChunk / kPer)) == 0 && ci * kChunk < n) part[ci] = c;
    uint32_t w = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) w += (uint32_t)__shfl_xor((int)w, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) t += wsum[k];
        sup[blockIdx.x] = t;
        atomicAdd(total, t);
    }
}

// Banded: the same chunk counts per band.  A position's tiles in band b are
// its rectangle's rows inside the band; the per-(band, chunk) sums gather in
// LDS, and each block adds its per-band sums to band_cnt.
__global__ void __launch_bounds__(kThreads) k_chunk_counts_banded(const JobDev* __restrict__ jobs, int n_jobs,
                                                                  const uint32_t* __restrict__ rects,
                                                                  const uint32_t* __restrict__ order, int64_t n,
                                                                  int nb, uint32_t* __restrict__ counts,
                                                                  uint32_t* __restrict__ band_cnt,
                                                                  uint32_t* __restrict__ total) {
    constexpr int kPer = kSuperChunk / kThreads;       // 16 consecutive positions per thread
    constexpr int kChunks = kSuperChunk / kChunk;      // 16 chunks per block
    __shared__ uint32_t s_cnt[kMaxBands * kChunks];
    __shared__ uint32_t wsum[kWaves];
    for (int e = threadIdx.x; e < nb * kChunks; e += kThreads) s_cnt[e] = 0u;
    __syncthreads();
    const int64_t first = (int64_t)blockIdx.x * kSuperChunk + (int64_t)threadIdx.x * kPer;
    const int chunk = threadIdx.x / (kChunk / kPer);
    uint32_t r[kPer], g[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        r[k] = first + k < n ? rects[first + k] : kEmptyRect;
        g[k] = first + k < n ? order[first + k] : 0u;
    }
    uint32_t sum = 0;
    for (int k = 0; k < kPer; ++k) {
        const uint32_t t = rect_tiles(r[k]);
        if (t == 0) continue;
        sum += t;
        const int j = find_job_gauss(jobs, n_jobs, (int64_t)g[k]);
        const int R = jobs[j].band_rows, B0 = jobs[j].band0;
        const int y0 = (r[k] >> 8) & 0xFF, y1 = r[k] >> 24;
        for (int kb = y0 / R; kb <= y1 / R; ++kb) {
            int lo, hi, w;
            band_rect(r[k], kb, R, lo, hi, w);
            if (hi >= lo) atomicAdd(&s_cnt[(B0 + kb) * kChunks + chunk], (uint32_t)((hi - lo + 1) * w));
        }
    }
    uint32_t ws = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) ws += (uint32_t)__shfl_xor((int)ws, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = ws;
    __syncthreads();
    const int64_t nchunk = (n + kChunk - 1) / kChunk;
    const int64_t words = chunk_count_words(n);
    for (int e = threadIdx.x; e < nb * kChunks; e += kThreads) {
        const int b = e / kChunks;
        const int64_t ci = (int64_t)blockIdx.x * kChunks + e % kChunks;
        if (ci < nchunk) counts[b * words + ci] = s_cnt[e];
    }
    if (threadIdx.x < nb) {
        const int b = threadIdx.x;
        uint32_t t = 0;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) t += s_cnt[b * kChunks + c];
        counts[b * words + nchunk + blockIdx.x] = t;
        if (t) atomicAdd(&band_cnt[b], t);
    }
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) t += wsum[k];
        atomicAdd(total, t);
    }
}

// Per band (one workgroup each): the 4096-position counts become their
// exclusive prefix over the depth order, in place, so an emission block
// finds its first position in a band's run with one load.
__global__ void __launch_bounds__(1024) k_band_sup_scan(uint32_t* __restrict__ counts, int64_t n) {
    __shared__ uint32_t scr[1024 / 64 + 1];
    const int64_t words = chunk_count_words(n);
    const int64_t nchunk = (n + kChunk - 1) / kChunk;
    const int64_t nsup = (n + kSuperChunk - 1) / kSuperChunk;
    uint32_t* sup = counts + blockIdx.x * words + nchunk;
    const int64_t per = (nsup + 1023) / 1024;
    const int64_t s0 = (int64_t)threadIdx.x * per < nsup ? (int64_t)threadIdx.x * per : nsup;
    const int64_t s1 = s0 + per < nsup ? s0 + per : nsup;
    uint32_t sum = 0;
    for (int64_t k = s0; k < s1; ++k) sum += sup[k];
    uint32_t total;
    uint32_t run = block_excl_scan<1024 / 64>(sum, scr, total);
    for (int64_t k = s0; k < s1; ++k) {
        const uint32_t v = sup[k];
        sup[k] = run;
        run += v;
    }
}

hipError_t launch_chunk_counts_banded(const JobDev* jobs, int n_jobs, const uint32_t* rects, const uint32_t* order,
                                      int64_t n, int nb, uint32_t* counts, uint32_t* band_cnt, uint32_t* total,
                                      hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (nb < 1 || nb > kMaxBands) return hipErrorInvalidValue;
    const int64_t nsup = (n + kSuperChunk - 1) / kSuperChunk;
    hipLaunchKernelGGL(k_chunk_counts_banded, dim3((unsigned)nsup), dim3(kThreads), 0, st, jobs, n_jobs, rects, order,
                       n, nb, counts, band_cnt, total);
    hipLaunchKernelGGL(k_band_sup_scan, dim3((unsigned)nb), dim3(1024), 0, st, counts, n);
    return hipGetLastError();
}


hipError_t launch_chunk_counts(const uint32_t* rects, const uint32_t* order, const uint32_t* touched, int64_t n,
                               uint32_t* counts, uint32_t* total, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int64_t nsup = (n + kSuperChunk - 1) / kSuperChunk;
    uint32_t* part = counts;
    uint32_t* sup = counts + (n + kChunk - 1) / kChunk;
    if (touched)
        hipLaunchKernelGGL(k_chunk_counts<true>, dim3((unsigned)nsup), dim3(kThreads), 0, st, rects, order, touched, n,
                           part, sup, total);
    else
        hipLaunchKernelGGL(k_chunk_counts<false>, dim3((unsigned)nsup), dim3(kThreads), 0, st, rects, order, touched,
                           n, part, sup, total);
    return hipGetLastError();
}

}  // namespace gs
