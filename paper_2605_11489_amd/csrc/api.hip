// C ABI of the rasterizer: argument checks, workspace layout and the launch
// sequence of the forward and backward passes.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gs3.h"
#include "gs_kernels.hpp"

namespace gs {

static_assert(kOverlapSquare == GS_OVERLAP_SQUARE && kOverlapOpacity == GS_OVERLAP_OPACITY &&
                  kOverlapEllipse == GS_OVERLAP_ELLIPSE,
              "overlap modes");

thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define GS_HIP_CHECK(expr)                                                                        \
    do {                                                                                          \
        hipError_t _e = (expr);                                                                   \
        if (_e != hipSuccess)                                                                     \
            return set_error(GS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));          \
    } while (0)

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int validate_job(const gs_job& j, int idx, bool need_outputs) {
    const gs_scene& s = j.scene;
    if (s.n < 0 || s.n > (int64_t)1 << 30)
        return set_error(GS_ERR_INVALID_ARG, "job %d: scene.n=%lld out of range", idx, (long long)s.n);
    if (s.sh_degree < 0 || s.sh_degree > GS_MAX_SH_DEGREE)
        return set_error(GS_ERR_INVALID_ARG, "job %d: sh_degree=%d not in 0..3", idx, s.sh_degree);
    if (s.n > 0 && (!s.means || !s.log_scales || !s.quats || !s.opacity_logits || !s.sh))
        return set_error(GS_ERR_INVALID_ARG, "job %d: null scene array", idx);
    if (s.n > 0 && ((uintptr_t)s.quats % 16) != 0)
        return set_error(GS_ERR_INVALID_ARG, "job %d: quats must be 16-byte aligned", idx);
    const int K3 = (s.sh_degree + 1) * (s.sh_degree + 1) * 3;
    if (s.n > 0 && (K3 % 4) == 0 && ((uintptr_t)s.sh % 16) != 0)
        return set_error(GS_ERR_INVALID_ARG, "job %d: sh must be 16-byte aligned", idx);
    const gs_camera& c = j.cam;
    if (c.width < 1 || c.height < 1 || c.width > 4096 || c.height > 4096)
        return set_error(GS_ERR_INVALID_ARG, "job %d: raster %dx%d out of range", idx, c.width, c.height);
    if (!(c.fx > 0) || !(c.fy > 0) || !isfinite(c.cx) || !isfinite(c.cy))
        return set_error(GS_ERR_INVALID_ARG, "job %d: invalid intrinsics", idx);
    for (int k = 0; k < 9; ++k)
        if (!isfinite(c.R_wc[k])) return set_error(GS_ERR_INVALID_ARG, "job %d: non-finite R_wc", idx);
    for (int k = 0; k < 3; ++k)
        if (!isfinite(c.t[k])) return set_error(GS_ERR_INVALID_ARG, "job %d: non-finite t", idx);
    if (!(j.opts.near_z > 0) || !(j.opts.dilation >= 0))
        return set_error(GS_ERR_INVALID_ARG, "job %d: near_z must be > 0 and dilation >= 0", idx);
    if (j.opts.overlap != GS_OVERLAP_SQUARE && j.opts.overlap != GS_OVERLAP_OPACITY &&
        j.opts.overlap != GS_OVERLAP_ELLIPSE)
        return set_error(GS_ERR_INVALID_ARG, "job %d: unknown overlap mode %d", idx, j.opts.overlap);
    if (need_outputs && (!j.out.final_T || !j.out.n_contrib))
        return set_error(GS_ERR_INVALID_ARG, "job %d: final_T and n_contrib are required", idx);
    return GS_OK;
}

// counters region: the words listed beside kCounterWords (pair count,
// capacity flag, compositing queue head, per-frame tiles done, per-band pairs)
static_assert(kBandCountWord - kJobDoneWord >= GS_MAX_BATCH, "a done count per frame");
constexpr size_t kCounterBytes = (size_t)kCounterWords * 4;

int tile_sort_bits(int64_t n_tiles) {
    int bits = 1;
    while (((int64_t)1 << bits) < n_tiles) ++bits;
    return bits;
}

// Whether a frame of the batch lists the exact ellipse tiles (then the pair
// counts and the emission take the projection's per-Gaussian counts).
inline bool any_ellipse(const gs_job* jobs, int n_jobs) {
    for (int j = 0; j < n_jobs; ++j)
        if (jobs[j].opts.overlap == GS_OVERLAP_ELLIPSE) return true;
    return false;
}

}  // namespace

// Tile bands of a batch over 2048 tiles (see BandDesc): frames of at most
// 2048 tiles are packed whole into bands, in batch order; a larger frame
// gets bands of floor(2048 / tiles_x) tile rows of its own.  nb == 0 when
// the batch has at most 2048 tiles (one ordinary pass), lists ellipse
// tiles, or would need more than kMaxBands bands (then the tile sort takes
// two passes and a boundary scan).
struct Bands {
    int nb = 0;
    int bits = 0;                       // digit bits of the banded pass
    uint32_t tile0[kMaxBands] = {};
    uint32_t ntiles[kMaxBands] = {};
    int32_t band0[GS_MAX_BATCH] = {};
    int32_t rows[GS_MAX_BATCH] = {};
    int32_t btile0[GS_MAX_BATCH] = {};
};

Bands plan_bands(const gs_job* jobs, int n_jobs) {
    Bands B;
    int64_t nt = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const int64_t tx = (jobs[j].cam.width + kTile - 1) / kTile, ty = (jobs[j].cam.height + kTile - 1) / kTile;
        B.band0[j] = 0;
        B.rows[j] = (int32_t)ty;
        B.btile0[j] = (int32_t)nt;
        nt += tx * ty;
    }
    if (nt <= kRsMaxBins || any_ellipse(jobs, n_jobs)) return B;
    Bands P = B;
    int nb = 0;
    bool open = false;
    int64_t tb = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const int64_t tx = (jobs[j].cam.width + kTile - 1) / kTile, ty = (jobs[j].cam.height + kTile - 1) / kTile;
        const int64_t T = tx * ty;
        if (T <= kRsMaxBins) {
            if (open && P.ntiles[nb - 1] + T <= (uint32_t)kRsMaxBins) {
                P.ntiles[nb - 1] += (uint32_t)T;
            } else {
                if (nb == kMaxBands) return B;
                P.tile0[nb] = (uint32_t)tb;
                P.ntiles[nb] = (uint32_t)T;
                ++nb;
                open = true;
            }
            P.band0[j] = nb - 1;
            P.rows[j] = (int32_t)ty;
            P.btile0[j] = (int32_t)P.tile0[nb - 1];
        } else {
            open = false;
            const int64_t R = kRsMaxBins / tx;   // tiles_x <= 256, so at least 8 rows
            const int64_t k = (ty + R - 1) / R;
            if (nb + k > kMaxBands) return B;
            P.band0[j] = nb;
            P.rows[j] = (int32_t)R;
            P.btile0[j] = (int32_t)tb;
            for (int64_t q = 0; q < k; ++q) {
                P.tile0[nb + q] = (uint32_t)(tb + q * R * tx);
                P.ntiles[nb + q] = (uint32_t)(((ty - q * R) < R ? (ty - q * R) : R) * tx);
            }
            nb += (int)k;
        }
        tb += T;
    }
    P.nb = nb;
    uint32_t most = 1;
    for (int b = 0; b < nb; ++b) most = std::max(most, P.ntiles[b]);
    P.bits = tile_sort_bits(most);
    return P;
}

int compute_layout(const gs_job* jobs, int n_jobs, int64_t key_capacity, int with_backward, gs_ws_layout* L,
                   bool need_outputs) {
    if (!jobs || !L) return set_error(GS_ERR_INVALID_ARG, "null jobs or layout");
    if (n_jobs < 1 || n_jobs > GS_MAX_BATCH)
        return set_error(GS_ERR_INVALID_ARG, "n_jobs=%d not in 1..%d", n_jobs, GS_MAX_BATCH);
    if (key_capacity < 0 || key_capacity > ((int64_t)1 << 31))
        return set_error(GS_ERR_INVALID_ARG, "key_capacity=%lld out of range", (long long)key_capacity);
    memset(L, 0, sizeof(*L));
    int64_t nf = 0, nt = 0;
    for (int j = 0; j < n_jobs; ++j) {
        int rc = validate_job(jobs[j], j, need_outputs);
        if (rc) return rc;
        L->gauss_base[j] = nf;
        L->tile_base[j] = nt;
        nf += (int64_t)align_up((size_t)jobs[j].scene.n, kGaussAlign);
        const int64_t tx = (jobs[j].cam.width + kTile - 1) / kTile;
        const int64_t ty = (jobs[j].cam.height + kTile - 1) / kTile;
        nt += tx * ty;
    }
    if (nt >= ((int64_t)1 << 31)) return set_error(GS_ERR_INVALID_ARG, "too many tiles");
    L->n_flat = nf;
    L->n_tiles = nt;
    L->key_capacity = key_capacity;
    size_t off = align_up(sizeof(JobDev) * kMaxJobs, 256);
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L->records = take((size_t)nf * sizeof(GaussRec));
    L->depth_keys = take((size_t)nf * 4);
    L->rects = take((size_t)nf * 4);
    L->touched = take((size_t)nf * 4);
    L->depth_order = take((size_t)nf * 4);
    L->depth_rects = take((size_t)nf * 4);
    const Bands B = plan_bands(jobs, n_jobs);
    L->chunk_counts = take((size_t)chunk_count_words(nf) * 4 * (size_t)std::max(B.nb, 1));
    L->tile_keys = take((size_t)key_capacity * 4);
    L->tile_values = take((size_t)key_capacity * 4);
    L->ranges = take((size_t)nt * 8);
    L->counters = take(kCounterBytes);
    L->grads2d = 0;
    bool normals = false;
    for (int j = 0; j < n_jobs; ++j) normals = normals || jobs[j].out.normal || jobs[j].out.nv;
    L->normals = normals ? take((size_t)nf * 16) : 0;
    L->total_bytes = off;
    return GS_OK;
}

// Scratch regions that are not part of the public layout (sort ping-pong,
// histograms) live after total_bytes of the public layout.
struct Scratch {
    size_t dk_a, dv_a, dr_a, dk_b, dv_b, dr_b;   // depth sort ping-pong (keys, indices, rectangles)
    size_t tk_e, tv_e, tk_t, tv_t;   // tile sort: emitted pairs and second buffer
    size_t hist, totals;
    size_t total;
    Bands bands;                     // tile bands (nb == 0: none)
};

// Appends the scratch regions (and the backward's per-Gaussian gradient
// buffer when asked) after the public regions; sets L->total_bytes.
Scratch compute_scratch(gs_ws_layout& L, int with_backward, const Bands& B) {
    Scratch S;
    S.bands = B;
    size_t off = L.total_bytes;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t nf = (size_t)L.n_flat, kc = (size_t)L.key_capacity;
    S.dk_a = take(nf * 4);
    S.dv_a = take(nf * 4);
    S.dr_a = take(nf * 4);
    S.dk_b = take(nf * 4);
    S.dv_b = take(nf * 4);
    S.dr_b = take(nf * 4);
    S.tk_e = take(kc * 4 + 16);   // 16-bit tile ids when one pass sorts them (read in aligned quads), else 32-bit
    S.tv_e = take(kc * 4);
    const int bits = tile_sort_bits(L.n_tiles);
    const bool two = bits > kRsMaxBits && B.nb == 0;
    S.tk_t = two ? take(kc * 4) : 0;
    S.tv_t = two ? take(kc * 4) : 0;
    const int64_t tile_hist = B.nb ? seg_hist_bytes((int64_t)kc, B.nb) : rs_hist_bytes((int64_t)kc);
    S.hist = take((size_t)std::max(rs_hist_bytes((int64_t)nf), tile_hist));
    S.totals = take((size_t)kRsMaxBins * 4 * std::max(B.nb, 1));
    L.grads2d = with_backward ? take(nf * 10 * 4) : 0;
    S.total = off;
    L.total_bytes = off;
    return S;
}

int plan(const gs_job* jobs, int n_jobs, int64_t key_capacity, int with_backward, bool need_outputs,
         gs_ws_layout* L, Scratch* S) {
    int rc = compute_layout(jobs, n_jobs, key_capacity, with_backward, L, need_outputs);
    if (rc) return rc;
    *S = compute_scratch(*L, with_backward, plan_bands(jobs, n_jobs));
    return GS_OK;
}

void fill_jobdev(const gs_job* jobs, int n_jobs, const gs_ws_layout& L, JobDev* out) {
    const Bands B = plan_bands(jobs, n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
        const gs_job& s = jobs[j];
        JobDev d;
        memset(&d, 0, sizeof(d));
        d.means = s.scene.means;
        d.log_scales = s.scene.log_scales;
        d.quats = s.scene.quats;
        d.opac = s.scene.opacity_logits;
        d.sh = s.scene.sh;
        d.n = s.scene.n;
        d.gauss_base = L.gauss_base[j];
        d.sh_degree = s.scene.sh_degree;
        d.tile_base = (int32_t)L.tile_base[j];
        d.width = s.cam.width;
        d.height = s.cam.height;
        d.tiles_x = (s.cam.width + kTile - 1) / kTile;
        d.tiles_y = (s.cam.height + kTile - 1) / kTile;
        memcpy(d.R, s.cam.R_wc, sizeof(d.R));
        memcpy(d.t, s.cam.t, sizeof(d.t));
        d.fx = s.cam.fx;
        d.fy = s.cam.fy;
        d.cx = s.cam.cx;
        d.cy = s.cam.cy;
        d.near_z = s.opts.near_z;
        d.dilation = s.opts.dilation;
        d.bg[0] = s.opts.bg[0];
        d.bg[1] = s.opts.bg[1];
        d.bg[2] = s.opts.bg[2];
        d.overlap = s.opts.overlap;
        d.band0 = B.band0[j];
        d.band_rows = B.rows[j];
        d.band_tile0 = B.btile0[j];
        d.rgb = s.out.rgb;
        d.alpha = s.out.alpha;
        d.depth = s.out.depth;
        d.dcdx = s.out.dcdx;
        d.dcdy = s.out.dcdy;
        d.final_T = s.out.final_T;
        d.n_contrib = s.out.n_contrib;
        d.n_evaluated = s.out.n_evaluated;
        d.n_blended = s.out.n_blended;
        d.normal = s.out.normal;
        d.nv = s.out.nv;
        out[j] = d;
    }
}

using u32 = uint32_t;

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}

// ------------------------------------------------------------ instrumentation
struct Profiler {
    bool active = false;
    int max_frames = 0;
    int frames = 0;
    int every = 1;
    int64_t passes = 0;   // forward passes seen since start
    std::vector<hipEvent_t> ev;   // (kStages + 1) events per recorded pass
    std::mutex mu;
};
constexpr int kStages = GS_N_STAGES;
Profiler g_prof;

// Event slot for boundary b of the current pass, or nullptr when not recording.
struct PassEvents {
    hipEvent_t e[kStages + 1];
    bool on = false;
};

PassEvents profile_pass() {
    PassEvents p;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!g_prof.active || g_prof.frames >= g_prof.max_frames) return p;
    if (g_prof.passes++ % g_prof.every != 0) return p;
    for (int b = 0; b <= kStages; ++b) p.e[b] = g_prof.ev[(size_t)g_prof.frames * (kStages + 1) + b];
    ++g_prof.frames;
    p.on = true;
    return p;
}

inline void mark(const PassEvents& p, int b, hipStream_t st) {
    if (p.on) (void)hipEventRecord(p.e[b], st);
}

// Projection, depth sort and the key-offset scan (shared by the forward pass
// and the key count query).
int run_front(const gs_job* jobs, int n_jobs, const gs_ws_layout& L, const Scratch& S, void* ws, hipStream_t st,
              const PassEvents& pe) {
    JobDev hj[GS_MAX_BATCH];
    fill_jobdev(jobs, n_jobs, L, hj);
    JobDev* dj = at<JobDev>(ws, 0);
    uint32_t* counters = at<uint32_t>(ws, L.counters);
    // the job table goes to the device and the counters (band counts
    // included) are cleared: by the projection itself for a single frame,
    // else by an upload launch before it
    const int n_zero = kBandCountWord + S.bands.nb;
    float4* nrm = L.normals ? at<float4>(ws, L.normals) : nullptr;
    if (n_jobs == 1) {
        mark(pe, 0, st);
        GS_HIP_CHECK(launch_project_one(hj[0], dj, counters, n_zero, L.n_flat, at<GaussRec>(ws, L.records),
                                        at<uint32_t>(ws, L.depth_keys), at<uint32_t>(ws, L.rects),
                                        at<uint32_t>(ws, L.touched), nrm, st));
    } else {
        GS_HIP_CHECK(launch_upload_jobs(hj, n_jobs, dj, st, counters, n_zero));
        mark(pe, 0, st);
        GS_HIP_CHECK(launch_project(dj, n_jobs, L.n_flat, at<GaussRec>(ws, L.records),
                                    at<uint32_t>(ws, L.depth_keys), at<uint32_t>(ws, L.rects),
                                    at<uint32_t>(ws, L.touched), nrm, st));
    }
    mark(pe, 1, st);
    const DevCount nf{nullptr, L.n_flat};
    uint32_t* hist = at<uint32_t>(ws, S.hist);
    uint32_t* tot = at<uint32_t>(ws, S.totals);
    // depth sort of all flat Gaussians by their 32-bit view-z key (passes of
    // 11, 11 and 10 bits); the packed tile rectangles move with the keys, so
    // the chunk counts and the emission read them in depth order without
    // gathers
    u32* dk_a = at<u32>(ws, S.dk_a);
    u32* dv_a = at<u32>(ws, S.dv_a);
    u32* dr_a = at<u32>(ws, S.dr_a);
    u32* dk_b = at<u32>(ws, S.dk_b);
    u32* dv_b = at<u32>(ws, S.dv_b);
    u32* dr_b = at<u32>(ws, S.dr_b);
    GS_HIP_CHECK(radix_pass(at<u32>(ws, L.depth_keys), nullptr, at<u32>(ws, L.rects), dk_a, dv_a, dr_a, nf, 0, 11,
                            hist, tot, nullptr, 0, st));
    GS_HIP_CHECK(radix_pass(dk_a, dv_a, dr_a, dk_b, dv_b, dr_b, nf, 11, 11, hist, tot, nullptr, 0, st));
    GS_HIP_CHECK(radix_pass(dk_b, dv_b, dr_b, nullptr, at<u32>(ws, L.depth_order), at<u32>(ws, L.depth_rects), nf,
                            22, 10, hist, tot, nullptr, 0, st));
    mark(pe, 2, st);
    // tile counts of depth-order chunks (per tile band when the tile sort is
    // banded); their total, the pair count, goes to counters[0]
    if (S.bands.nb)
        GS_HIP_CHECK(launch_chunk_counts_banded(dj, n_jobs, at<u32>(ws, L.depth_rects), at<u32>(ws, L.depth_order),
                                                L.n_flat, S.bands.nb, at<u32>(ws, L.chunk_counts),
                                                counters + kBandCountWord, counters, st));
    else
        GS_HIP_CHECK(launch_chunk_counts(at<u32>(ws, L.depth_rects), at<u32>(ws, L.depth_order),
                                         any_ellipse(jobs, n_jobs) ? at<u32>(ws, L.touched) : nullptr, L.n_flat,
                                         at<u32>(ws, L.chunk_counts), counters, st));
    return GS_OK;
}

// Where the work-queue compositing publishes each frame's completion.
struct DoneSignal {
    uint32_t* host;   // one word per frame, host memory
    uint32_t seq;
};

// Emission, tile sort, tile ranges and compositing (after run_front); with
// `done` and more than one frame, the compositing is the persistent
// work-queue kernel, which publishes each frame but the last as it completes.
int run_back(const gs_job* jobs, int n_jobs, const gs_ws_layout& L, const Scratch& S, void* ws,
             int64_t key_capacity, hipStream_t st, const PassEvents& pe, const DoneSignal* done = nullptr) {
    uint32_t* counters = at<uint32_t>(ws, L.counters);
    JobDev* dj = at<JobDev>(ws, 0);
    const Bands& B = S.bands;
    if (B.nb)
        GS_HIP_CHECK(launch_emit_banded(dj, n_jobs, L.n_flat, at<uint32_t>(ws, L.depth_order),
                                        at<uint32_t>(ws, L.chunk_counts), at<uint32_t>(ws, L.depth_rects), B.nb,
                                        counters + kBandCountWord, at<uint16_t>(ws, S.tk_e),
                                        at<uint32_t>(ws, S.tv_e), key_capacity, counters, st));
    else
        GS_HIP_CHECK(launch_emit(dj, n_jobs, L.n_flat, at<uint32_t>(ws, L.depth_order),
                                 at<uint32_t>(ws, L.chunk_counts), at<uint32_t>(ws, L.depth_rects),
                                 any_ellipse(jobs, n_jobs) ? at<uint32_t>(ws, L.touched) : nullptr,
                                 at<GaussRec>(ws, L.records), at<uint32_t>(ws, S.tk_e),
                                 tile_sort_bits(L.n_tiles) <= kRsMaxBits, at<uint32_t>(ws, S.tv_e), key_capacity,
                                 counters, st));
    mark(pe, 3, st);
    // stable sort of the pairs by global tile id; in one pass (up to 2048
    // tiles) the digit starts are the tile ranges, written by the sort itself
    const DevCount nk{counters, key_capacity};
    const int bits = tile_sort_bits(L.n_tiles);
    const int passes = (bits + kRsMaxBits - 1) / kRsMaxBits;
    const int per = (bits + passes - 1) / passes;
    uint32_t* hist = at<uint32_t>(ws, S.hist);
    uint32_t* tot = at<uint32_t>(ws, S.totals);
    uint32_t* src_k = at<uint32_t>(ws, S.tk_e);
    uint32_t* src_v = at<uint32_t>(ws, S.tv_e);
    if (B.nb) {
        // one stable pass per band's run, on band-local tile ids
        BandDesc bd;
        memset(&bd, 0, sizeof(bd));
        bd.cnt = counters + kBandCountWord;
        bd.cap = key_capacity;
        bd.nb = B.nb;
        memcpy(bd.tile0, B.tile0, sizeof(bd.tile0));
        memcpy(bd.ntiles, B.ntiles, sizeof(bd.ntiles));
        GS_HIP_CHECK(radix_pass_banded(at<uint16_t>(ws, S.tk_e), src_v, at<uint32_t>(ws, L.tile_values), bd, B.bits,
                                       hist, tot, at<uint32_t>(ws, L.ranges), st));
    } else if (passes == 1) {
        GS_HIP_CHECK(radix_pass_tiles(at<uint16_t>(ws, S.tk_e), src_v, at<uint32_t>(ws, L.tile_values), nk, bits,
                                      hist, tot, at<uint32_t>(ws, L.ranges), L.n_tiles, st));
    } else {
        for (int p = 0; p < passes; ++p) {
            const bool lastp = p == passes - 1;
            uint32_t* dk = lastp ? at<uint32_t>(ws, L.tile_keys)
                                 : (p % 2 == 0 ? at<uint32_t>(ws, S.tk_t) : at<uint32_t>(ws, S.tk_e));
            uint32_t* dv = lastp ? at<uint32_t>(ws, L.tile_values)
                                 : (p % 2 == 0 ? at<uint32_t>(ws, S.tv_t) : at<uint32_t>(ws, S.tv_e));
            const int b = (p * per + per <= bits) ? per : bits - p * per;
            GS_HIP_CHECK(radix_pass(src_k, src_v, nullptr, dk, dv, nullptr, nk, p * per, b, hist, tot, nullptr, 0, st));
            src_k = dk;
            src_v = dv;
        }
        GS_HIP_CHECK(launch_ranges(at<uint32_t>(ws, L.tile_keys), nk, at<uint32_t>(ws, L.ranges), L.n_tiles, st));
    }
    mark(pe, 4, st);
    bool count = false;
    for (int j = 0; j < n_jobs; ++j) count = count || jobs[j].out.n_evaluated || jobs[j].out.n_blended;
    // (a single frame is complete when its batch is: the plain grid is the
    // faster one there)
    if (done && n_jobs > 1)
        GS_HIP_CHECK(launch_composite_queue(dj, n_jobs, L.n_tiles, L.n_flat, at<GaussRec>(ws, L.records),
                                            at<uint32_t>(ws, L.tile_values), at<uint32_t>(ws, L.ranges),
                                            L.key_capacity, counters, done->host, done->seq, st));
    else
        GS_HIP_CHECK(launch_composite(dj, n_jobs, L.n_tiles, L.n_flat, at<GaussRec>(ws, L.records),
                                  at<uint32_t>(ws, L.tile_values), at<uint32_t>(ws, L.ranges), L.key_capacity,
                                  count, L.normals ? at<float4>(ws, L.normals) : nullptr, st));
    mark(pe, 5, st);
    return GS_OK;
}

int check_workspace(void* ws, size_t ws_bytes, const Scratch& S) {
    if (!ws) return set_error(GS_ERR_INVALID_ARG, "null workspace");
    if (ws_bytes < S.total)
        return set_error(GS_ERR_INVALID_ARG, "workspace of %zu bytes < required %zu", ws_bytes, S.total);
    if (((uintptr_t)ws % 256) != 0) return set_error(GS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    return GS_OK;
}

int run_forward(const gs_job* jobs, int n_jobs, void* ws, size_t ws_bytes, int64_t key_capacity, hipStream_t st,
                int with_backward, const DoneSignal* done = nullptr) {
    gs_ws_layout L;
    Scratch S;
    int rc = plan(jobs, n_jobs, key_capacity, with_backward, true, &L, &S);
    if (rc) return rc;
    if ((rc = check_workspace(ws, ws_bytes, S))) return rc;
    const PassEvents pe = profile_pass();
    rc = run_front(jobs, n_jobs, L, S, ws, st, pe);
    if (rc) return rc;
    return run_back(jobs, n_jobs, L, S, ws, key_capacity, st, pe, done);
}

// A server batch's forward pass (the serving loop's only launch path): as
// gs_render_forward_batch, with the compositing of a batch of several frames
// done by the persistent work-queue kernel, which stores seq into
// done_host[j] (host memory, one word per frame) as soon as frame j is
// complete, for every frame but the batch's last.  Counting and normal
// outputs are not supported here (the server never asks for them).
int render_forward_signalled(const gs_job* jobs, int n_jobs, void* ws, size_t ws_bytes, int64_t key_capacity,
                             uint32_t* done_host, uint32_t seq, hipStream_t st) {
    if (!done_host) return set_error(GS_ERR_INVALID_ARG, "null completion words");
    for (int j = 0; j < n_jobs; ++j)
        if (jobs[j].out.n_evaluated || jobs[j].out.n_blended || jobs[j].out.normal || jobs[j].out.nv)
            return set_error(GS_ERR_INVALID_ARG, "job %d: counting and normal outputs are not served", j);
    const DoneSignal done{done_host, seq};
    return run_forward(jobs, n_jobs, ws, ws_bytes, key_capacity, st, 0, &done);
}

// Per host thread and device: a pinned word that receives a frame's pair
// count and an event marking its arrival (created on first use).
struct CountSync {
    hipEvent_t ev = nullptr;
    uint32_t* host = nullptr;
};

int count_sync(CountSync** out) {
    thread_local std::vector<CountSync> per_device;
    int dev = 0;
    GS_HIP_CHECK(hipGetDevice(&dev));
    if ((int)per_device.size() <= dev) per_device.resize(dev + 1);
    CountSync& c = per_device[dev];
    if (!c.ev) {
        GS_HIP_CHECK(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
        GS_HIP_CHECK(hipHostMalloc((void**)&c.host, 64, hipHostMallocDefault));
    }
    *out = &c;
    return GS_OK;
}

// The whole pass is launched; the host waits only until the pair count of
// the front half has reached pinned memory, while the device goes on with
// the back half.  A pass whose pairs exceed the capacity drops the extra
// pairs (every kernel stays within the capacity) and reports it.
int run_forward_checked(const gs_job* jobs, int n_jobs, void* ws, size_t ws_bytes, int64_t key_capacity,
                        int with_backward, int64_t* keys_needed, hipStream_t st) {
    gs_ws_layout L;
    Scratch S;
    int rc = plan(jobs, n_jobs, key_capacity, with_backward, true, &L, &S);
    if (rc) return rc;
    if ((rc = check_workspace(ws, ws_bytes, S))) return rc;
    CountSync* cs = nullptr;
    if ((rc = count_sync(&cs))) return rc;
    const PassEvents pe = profile_pass();
    rc = run_front(jobs, n_jobs, L, S, ws, st, pe);
    if (rc) return rc;
    GS_HIP_CHECK(hipMemcpyAsync(cs->host, at<uint32_t>(ws, L.counters), sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GS_HIP_CHECK(hipEventRecord(cs->ev, st));
    rc = run_back(jobs, n_jobs, L, S, ws, key_capacity, st, pe);
    if (rc) return rc;
    GS_HIP_CHECK(hipEventSynchronize(cs->ev));
    const uint32_t pairs = *cs->host;
    if (keys_needed) *keys_needed = (int64_t)pairs;
    if ((int64_t)pairs > key_capacity)
        return set_error(GS_ERR_CAPACITY, "frame needs %u keys, workspace holds %lld", pairs, (long long)key_capacity);
    return GS_OK;
}

// ------------------------------------------------------------ no-alloc forward
// The forward pass for callers that cannot allocate (code under graph
// capture, serving loops that forbid allocation): its workspace is this
// file-scope device array, one per GPU, held until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address of each GPU's copy is looked
// up once per device and kept in g_scratch_ptr.
constexpr size_t kNoAllocScratchBytes = (size_t)384 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_ptr(void** out) {
    int dev = 0;
    GS_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(GS_ERR_INVALID_ARG, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        GS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(GS_ERR_HIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GS_OK;
}

__global__ void k_copy_counts(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
    if (threadIdx.x < 2) dst[threadIdx.x] = src[threadIdx.x];
}

gs_job make_job(const gs_scene* scene, const gs_camera* cam, const gs_render_opts* opts, const gs_outputs* out) {
    gs_job j;
    memset(&j, 0, sizeof(j));
    j.scene = *scene;
    j.cam = *cam;
    j.opts = *opts;
    if (out) j.out = *out;
    return j;
}

}  // namespace gs

using namespace gs;

extern "C" {

int gs_forward_layout(const gs_job* jobs, int n_jobs, int64_t key_capacity, int with_backward,
                      gs_ws_layout* layout) {
    Scratch S;
    return plan(jobs, n_jobs, key_capacity, with_backward, false, layout, &S);
}

int gs_count_keys(const gs_job* jobs, int n_jobs, void* workspace, size_t ws_bytes, int64_t* keys_per_job,
                  void* stream) {
    if (!keys_per_job) return set_error(GS_ERR_INVALID_ARG, "null keys_per_job");
    gs_ws_layout L;
    Scratch S;
    int rc = plan(jobs, n_jobs, 0, 0, false, &L, &S);
    if (rc) return rc;
    if (!workspace || ws_bytes < S.total)
        return set_error(GS_ERR_INVALID_ARG, "workspace too small (%zu < %zu)", ws_bytes, S.total);
    hipStream_t st = (hipStream_t)stream;
    JobDev hj[GS_MAX_BATCH];
    fill_jobdev(jobs, n_jobs, L, hj);
    JobDev* dj = at<JobDev>(workspace, 0);
    GS_HIP_CHECK(launch_upload_jobs(hj, n_jobs, dj, st));
    GS_HIP_CHECK(launch_project(dj, n_jobs, L.n_flat, at<GaussRec>(workspace, L.records),
                                at<uint32_t>(workspace, L.depth_keys), at<uint32_t>(workspace, L.rects),
                                at<uint32_t>(workspace, L.touched), nullptr, st));
    std::vector<uint32_t> touched((size_t)L.n_flat);
    if (L.n_flat)
        GS_HIP_CHECK(hipMemcpyAsync(touched.data(), at<uint32_t>(workspace, L.touched), (size_t)L.n_flat * 4,
                                    hipMemcpyDeviceToHost, st));
    GS_HIP_CHECK(hipStreamSynchronize(st));
    for (int j = 0; j < n_jobs; ++j) {
        int64_t sum = 0;
        for (int64_t g = 0; g < jobs[j].scene.n; ++g) sum += touched[(size_t)(L.gauss_base[j] + g)];
        keys_per_job[j] = sum;
    }
    return GS_OK;
}

int gs_render_forward_batch(const gs_job* jobs, int n_jobs, void* workspace, size_t ws_bytes, int64_t key_capacity,
                            void* stream) {
    return run_forward(jobs, n_jobs, workspace, ws_bytes, key_capacity, (hipStream_t)stream, 0);
}

int gs_render_forward_checked(const gs_job* jobs, int n_jobs, void* workspace, size_t ws_bytes,
                              int64_t key_capacity, int with_backward, int64_t* keys_needed, void* stream) {
    return run_forward_checked(jobs, n_jobs, workspace, ws_bytes, key_capacity, with_backward, keys_needed,
                               (hipStream_t)stream);
}

int gs_render_forward_noalloc(const gs_job* jobs, int n_jobs, int64_t key_capacity, uint32_t* counts_out,
                              void* stream) {
    gs_ws_layout L;
    Scratch S;
    int rc = plan(jobs, n_jobs, key_capacity, 0, true, &L, &S);
    if (rc) return rc;
    if (S.total > kNoAllocScratchBytes)
        return set_error(GS_ERR_TOO_LARGE, "the frame's workspace (%zu bytes for %lld pairs) exceeds the %zu-byte "
                         "no-alloc scratch", S.total, (long long)key_capacity, kNoAllocScratchBytes);
    void* ws = nullptr;
    if ((rc = scratch_ptr(&ws))) return rc;
    hipStream_t st = (hipStream_t)stream;
    // every region the pass reads is written by the pass first (the counters
    // are cleared by its first kernel), so the array's previous contents,
    // left by the last call on this device, do not matter
    if ((rc = run_forward(jobs, n_jobs, ws, kNoAllocScratchBytes, key_capacity, st, 0))) return rc;
    if (counts_out) {
        hipLaunchKernelGGL(k_copy_counts, dim3(1), dim3(64), 0, st, at<const uint32_t>(ws, L.counters), counts_out);
        GS_HIP_CHECK(hipGetLastError());
    }
    return GS_OK;
}

int gs_render_forward(const gs_scene* scene, const gs_camera* cam, const gs_render_opts* opts,
                      const gs_outputs* out, void* workspace, size_t ws_bytes, int64_t key_capacity, void* stream) {
    if (!scene || !cam || !opts || !out) return set_error(GS_ERR_INVALID_ARG, "null argument");
    const gs_job j = make_job(scene, cam, opts, out);
    return run_forward(&j, 1, workspace, ws_bytes, key_capacity, (hipStream_t)stream, 0);
}

int gs_forward_status(const void* workspace, const gs_ws_layout* layout, int64_t* keys_needed) {
    if (!workspace || !layout) return set_error(GS_ERR_INVALID_ARG, "null argument");
    uint32_t c[4];
    GS_HIP_CHECK(hipMemcpy(c, reinterpret_cast<const char*>(workspace) + layout->counters, sizeof(c),
                           hipMemcpyDeviceToHost));
    if (keys_needed) *keys_needed = (int64_t)c[0];
    if (c[1] != 0u)
        return set_error(GS_ERR_CAPACITY, "frame needs %u keys, workspace holds %lld", c[0],
                         (long long)layout->key_capacity);
    return GS_OK;
}

int gs_sorted_keys(const gs_job* jobs, int n_jobs, int job, const void* workspace, const gs_ws_layout* layout,
                   uint64_t* keys_out, uint32_t* values_out, void* stream) {
    if (!workspace || !layout || !keys_out || !values_out) return set_error(GS_ERR_INVALID_ARG, "null argument");
    if (job < 0 || job >= n_jobs) return set_error(GS_ERR_INVALID_ARG, "job %d out of range", job);
    hipStream_t st = (hipStream_t)stream;
    const int64_t tiles = ((jobs[job].cam.width + kTile - 1) / kTile) * (int64_t)((jobs[job].cam.height + kTile - 1) / kTile);
    std::vector<uint32_t> rg((size_t)tiles * 2);
    void* ws = const_cast<void*>(workspace);
    GS_HIP_CHECK(hipMemcpyAsync(rg.data(), at<uint32_t>(ws, layout->ranges) + 2 * layout->tile_base[job],
                                rg.size() * 4, hipMemcpyDeviceToHost, st));
    GS_HIP_CHECK(hipStreamSynchronize(st));
    int64_t begin = -1, end = -1;
    for (int64_t t = 0; t < tiles; ++t) {
        if (rg[2 * t + 1] > rg[2 * t]) {
            if (begin < 0) begin = rg[2 * t];
            end = rg[2 * t + 1];
        }
    }
    if (begin < 0) return GS_OK;
    GS_HIP_CHECK(launch_compose_keys(at<uint32_t>(ws, layout->ranges) + 2 * layout->tile_base[job], tiles,
                                     at<uint32_t>(ws, layout->tile_values), at<uint32_t>(ws, layout->depth_keys),
                                     begin, layout->gauss_base[job], keys_out, values_out, st));
    return GS_OK;
}

int gs_gradient_upsample(const float* rgb, const float* dcdx, const float* dcdy, int32_t width, int32_t height,
                         int32_t scale, float* out, void* stream) {
    if (!rgb || !dcdx || !dcdy || !out) return set_error(GS_ERR_INVALID_ARG, "null buffer");
    if (width < 1 || width > 4096 || height < 1 || height > 4096)
        return set_error(GS_ERR_INVALID_ARG, "image %dx%d out of range 1..4096", width, height);
    if (scale < 1 || scale > 4) return set_error(GS_ERR_INVALID_ARG, "scale %d out of range 1..4", scale);
    GS_HIP_CHECK(launch_gradient_upsample(rgb, dcdx, dcdy, width, height, scale, out, (hipStream_t)stream));
    return GS_OK;
}

static int check_warp_camera(const gs_camera* c, const char* which) {
    if (!c) return set_error(GS_ERR_INVALID_ARG, "null %s camera", which);
    if (c->width < 1 || c->height < 1 || c->width > 4096 || c->height > 4096)
        return set_error(GS_ERR_INVALID_ARG, "%s raster %dx%d out of range 1..4096", which, c->width, c->height);
    if (!(c->fx > 0) || !(c->fy > 0) || !isfinite(c->fx) || !isfinite(c->fy) || !isfinite(c->cx) ||
        !isfinite(c->cy))
        return set_error(GS_ERR_INVALID_ARG, "%s camera: invalid intrinsics", which);
    for (int k = 0; k < 9; ++k)
        if (!isfinite(c->R_wc[k])) return set_error(GS_ERR_INVALID_ARG, "%s camera: non-finite R_wc", which);
    for (int k = 0; k < 3; ++k)
        if (!isfinite(c->t[k])) return set_error(GS_ERR_INVALID_ARG, "%s camera: non-finite t", which);
    return GS_OK;
}

static size_t warp_bytes(const gs_camera* src, const gs_camera* dst) {
    return warp_workspace_bytes((int64_t)src->width * src->height, (int64_t)dst->width * dst->height);
}

int gs_warp_workspace_size(const gs_camera* src, const gs_camera* dst, size_t* bytes) {
    if (!bytes) return set_error(GS_ERR_INVALID_ARG, "null bytes");
    if (int rc = check_warp_camera(src, "source")) return rc;
    if (int rc = check_warp_camera(dst, "destination")) return rc;
    *bytes = warp_bytes(src, dst);
    return GS_OK;
}

int gs_motion_warp(const gs_camera* src, const gs_camera* dst, const float* rgb, const float* alpha,
                   const float* depth, const float* dcdx, const float* dcdy, const float* normal, float* motion,
                   const gs_warp_outputs* out, void* workspace, size_t ws_bytes, void* stream) {
    if (int rc = check_warp_camera(src, "source")) return rc;
    if (int rc = check_warp_camera(dst, "destination")) return rc;
    if (!out) return set_error(GS_ERR_INVALID_ARG, "null outputs");
    if (!alpha || !depth) return set_error(GS_ERR_INVALID_ARG, "alpha and depth are required");
    if (out->rgb && !rgb) return set_error(GS_ERR_INVALID_ARG, "warped rgb asked for without source rgb");
    if ((out->dcdx || out->dcdy) && (!dcdx || !dcdy))
        return set_error(GS_ERR_INVALID_ARG, "warped gradients asked for without source dcdx and dcdy");
    if (out->normal && !normal) return set_error(GS_ERR_INVALID_ARG, "warped normals asked for without a normal map");
    if (!workspace || ws_bytes < warp_bytes(src, dst))
        return set_error(GS_ERR_INVALID_ARG, "workspace of %zu bytes, %zu needed", ws_bytes, warp_bytes(src, dst));
    if ((uintptr_t)workspace % 16 != 0) return set_error(GS_ERR_INVALID_ARG, "workspace must be 16-byte aligned");
    WarpCams c;
    for (int k = 0; k < 9; ++k) {
        c.Rs[k] = src->R_wc[k];
        c.Rd[k] = dst->R_wc[k];
    }
    for (int k = 0; k < 3; ++k) {
        c.ts[k] = src->t[k];
        c.td[k] = dst->t[k];
    }
    c.fxs = src->fx, c.fys = src->fy, c.cxs = src->cx, c.cys = src->cy;
    c.fxd = dst->fx, c.fyd = dst->fy, c.cxd = dst->cx, c.cyd = dst->cy;
    c.W = src->width, c.H = src->height, c.Wd = dst->width, c.Hd = dst->height;
    WarpOut o{out->rgb, out->depth, out->dcdx, out->dcdy, out->weight, out->source, out->normal};
    GS_HIP_CHECK(
        launch_motion_warp(c, rgb, alpha, depth, dcdx, dcdy, normal, motion, o, workspace, (hipStream_t)stream));
    return GS_OK;
}

int gs_profile_start(int max_frames, int every) {
    if (max_frames < 1 || max_frames > 1000000) return set_error(GS_ERR_INVALID_ARG, "max_frames out of range");
    if (every < 1 || every > 1000000) return set_error(GS_ERR_INVALID_ARG, "every out of range");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (hipEvent_t e : g_prof.ev) (void)hipEventDestroy(e);
    g_prof.ev.assign((size_t)max_frames * (kStages + 1), nullptr);
    for (auto& e : g_prof.ev) GS_HIP_CHECK(hipEventCreate(&e));
    g_prof.max_frames = max_frames;
    g_prof.frames = 0;
    g_prof.every = every;
    g_prof.passes = 0;
    g_prof.active = true;
    return GS_OK;
}

int gs_profile_stop(double* stage_ms, int64_t* frames) {
    if (!stage_ms || !frames) return set_error(GS_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!g_prof.active) return set_error(GS_ERR_INVALID_ARG, "profiling was not started");
    g_prof.active = false;
    for (int s = 0; s < kStages; ++s) stage_ms[s] = 0.0;
    for (int f = 0; f < g_prof.frames; ++f) {
        hipEvent_t* e = &g_prof.ev[(size_t)f * (kStages + 1)];
        GS_HIP_CHECK(hipEventSynchronize(e[kStages]));
        for (int s = 0; s < kStages; ++s) {
            float ms = 0.f;
            GS_HIP_CHECK(hipEventElapsedTime(&ms, e[s], e[s + 1]));
            stage_ms[s] += ms;
        }
    }
    *frames = g_prof.frames;
    return GS_OK;
}

int gs_render_backward(const gs_scene* scene, const gs_camera* cam, const gs_render_opts* opts,
                       const gs_outputs* fwd_out, void* workspace, size_t ws_bytes, int64_t key_capacity,
                       const float* dL_drgb, const float* dL_dalpha, const float* dL_ddepth, const gs_grads* grads,
                       void* stream) {
    if (!scene || !cam || !opts || !fwd_out || !grads || !dL_drgb)
        return set_error(GS_ERR_INVALID_ARG, "null argument");
    if (scene->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits ||
                         !grads->sh))
        return set_error(GS_ERR_INVALID_ARG, "null gradient array");
    if (scene->n > 0 && ((uintptr_t)grads->quats % 16) != 0)
        return set_error(GS_ERR_INVALID_ARG, "grads->quats must be 16-byte aligned");
    if (scene->n > 0 && (3 * (scene->sh_degree + 1) * (scene->sh_degree + 1)) % 4 == 0 &&
        ((uintptr_t)grads->sh % 16) != 0)
        return set_error(GS_ERR_INVALID_ARG, "grads->sh must be 16-byte aligned");
    const gs_job jb = make_job(scene, cam, opts, fwd_out);
    gs_ws_layout L;
    Scratch S;
    int rc = plan(&jb, 1, key_capacity, 1, true, &L, &S);
    if (rc) return rc;
    if (!workspace || ws_bytes < S.total)
        return set_error(GS_ERR_INVALID_ARG, "workspace of %zu bytes < %zu (size it with with_backward=1)", ws_bytes,
                         S.total);
    hipStream_t st = (hipStream_t)stream;
    void* ws = workspace;
    JobDev hj[1];
    fill_jobdev(&jb, 1, L, hj);
    JobDev* dj = at<JobDev>(ws, 0);
    float* g2 = at<float>(ws, L.grads2d);
    // the per-Gaussian gradient sums cleared and the job table written in one launch
    GS_HIP_CHECK(launch_fill_u32_job(reinterpret_cast<uint32_t*>(g2), 0u, L.n_flat * 10, hj[0], dj, st));
    GS_HIP_CHECK(launch_composite_bwd(dj, 1, L.n_tiles, L.n_flat, at<GaussRec>(ws, L.records),
                                      at<uint32_t>(ws, L.tile_values), at<uint32_t>(ws, L.ranges), dL_drgb, dL_dalpha,
                                      dL_ddepth, g2, st));
    GS_HIP_CHECK(launch_project_bwd(dj, 1, L.n_flat, at<uint32_t>(ws, L.touched), g2, grads->means,
                                    grads->log_scales, grads->quats, grads->opacity_logits, grads->sh,
                                    grads->overwrite != 0, st));
    return GS_OK;
}

const char* gs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
