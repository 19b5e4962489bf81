// Continuous-batching render server (the gs_server_* entry points).
//
// One worker thread owns the device side: it reaps finished batches (event
// queries, never a blocking wait), then forms new batches from the pending
// queue in arrival order as long as a stream slot and arena memory are free,
// and launches each batch as one gs_render_forward_batch on its slot's
// stream.  Frames of different scenes and resolutions share every launch of
// a batch; batches on different streams overlap on the device.  All memory
// (scenes, outputs, workspaces) comes from one arena reserved at creation,
// so admission is an exact check against the budget.
//
// Admission is cost-aware.  Every (scene, raster size) class keeps an
// estimate of its frame time (first from its pair count, then from the
// measured time of its single-frame batches).  A heavy frame (estimate at
// or above heavy_ms) starts once nothing else is on the device, and only
// tiny frames (a quarter of heavy_ms and below) start beside it, so sharing
// the GPU barely stretches the longest frames that set the tail.  Light
// frames are batched and overlap with each other; a heavy frame at the head
// of the queue holds back the frames behind it until it has started
// (arrival order is kept, so no frame starves).
//
// Within a batch the frames are ordered shortest first.  In work-queue mode
// a batch of several frames is composited by the persistent work-queue
// kernel, which stores the batch's sequence number into a frame's word of a
// pinned host array once the frame is complete; gs_poll and the worker read
// those words, so such a frame is done before the rest of its batch.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/gs3.h"
#include "gs_common.hpp"

namespace gs {
int set_error(int code, const char* fmt, ...);
int render_forward_signalled(const gs_job* jobs, int n_jobs, void* ws, size_t ws_bytes, int64_t key_capacity,
                             uint32_t* done_host, uint32_t seq, hipStream_t st);
}

using gs::set_error;

namespace {

double now_s() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing of freed neighbours.
struct Arena {
    size_t size = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_;   // offset -> length

    void init(size_t s) {
        size = s & ~(size_t)255;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t* off) {
        n = align256(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rem = it->second - n, o2 = it->first + n;
                free_.erase(it);
                if (rem) free_[o2] = rem;
                used += n;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = align256(n ? n : 1);
        used -= n;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + n == nx->first) {
            n += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += n;
                return;
            }
        }
        free_[off] = n;
    }
};

struct SceneRec {
    gs_scene scene;   // pointers into the arena
    size_t off = 0, bytes = 0;
};

struct Req {
    uint64_t ticket = 0;
    int32_t scene = 0;
    gs_camera cam;
    gs_render_opts opts;
    int status = GS_ERR_NOT_READY;
    bool finished = false;
    double t_submit = 0, t_start = 0, t_done = 0;
    size_t out_off = 0, out_bytes = 0;
    bool has_out = false;
    int64_t cap = 0;
    int retries = 0;
    int batch_size = 0;
    gs_outputs out;
    // while in flight: the slot and the frame's index in its batch, whose
    // completion word the compositing kernel sets to the batch's sequence number
    int slot = -1, job = -1;
    bool flag_done = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;         // end of the batch (timing enabled)
    hipEvent_t ev_start = nullptr;      // start of the batch
    uint32_t* counters_host = nullptr;   // pinned
    // pinned, coherent: word j receives `seq` from the compositing kernel
    // once frame j of the slot's batch is complete
    uint32_t* done_host = nullptr;
    uint32_t* done_dev = nullptr;        // the same words as the device addresses them
    uint32_t seq = 0;                    // the batch's sequence number (never 0)
    bool busy = false;
    bool heavy = false;                  // the batch is one heavy frame running alone
    std::vector<uint64_t> tickets;
    size_t ws_off = 0, ws_bytes = 0;
    int64_t cap = 0;
    double sim_done_at = 0;
    bool sim_fail = false;
};

// Frame-time estimate of one (scene, raster size) class.
struct ClassEst {
    int64_t keys = 0;    // pairs (largest seen)
    double ms = 0;       // frame time
    int samples = 0;     // measured single-frame batches folded into ms
};

// First estimate of a frame's time from its pair count and Gaussian count,
// before any frame of its class has been timed (slightly above the measured
// single-frame times of the rasterizer: 0.36 ms for 1M Gaussians and 10.8M
// pairs, 3.2 ms for 6M and 186M).
double model_ms(int64_t keys, int64_t n) { return 0.05 + 0.02e-6 * (double)keys + 0.06e-6 * (double)n; }

size_t out_bytes_for(int W, int H) { return (size_t)W * H * 13 * 4 + 13 * 256; }

}  // namespace

struct gs_server {
    gs_server_opts o;
    char* base = nullptr;   // device arena (nullptr when simulating)
    Arena arena;
    std::vector<SceneRec> scenes;
    size_t scene_bytes = 0;
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> pending;
    std::vector<Slot> slots;
    std::map<std::tuple<int, int, int>, ClassEst> key_est;   // (scene, W, H) -> estimates
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t st_submitted = 0, st_completed = 0, st_failed = 0, st_rejected = 0, st_batches = 0, st_maxbatch = 0;
    int64_t st_flag_done = 0;
    int64_t batch_counter = 0;
    hipStream_t probe_stream = nullptr;

    gs_outputs outputs_at(size_t off, int W, int H) {
        gs_outputs out;
        memset(&out, 0, sizeof(out));
        const size_t px = (size_t)W * H;
        size_t o = off;
        auto take = [&](size_t n) {
            char* p = base + o;
            o += align256(n);
            return p;
        };
        out.rgb = (float*)take(3 * px * 4);
        out.alpha = (float*)take(px * 4);
        out.depth = (float*)take(px * 4);
        out.dcdx = (float*)take(3 * px * 4);
        out.dcdy = (float*)take(3 * px * 4);
        out.final_T = (float*)take(px * 4);
        out.n_contrib = (uint32_t*)take(px * 4);
        return out;
    }

    gs_job job_for(const Req& r) {
        gs_job j;
        memset(&j, 0, sizeof(j));
        j.scene = scenes[r.scene].scene;
        j.cam = r.cam;
        j.opts = r.opts;
        j.out = r.out;
        return j;
    }

    // pairs estimate for a request's class; probes the first request of a class
    int64_t estimate_keys(const Req& r) {
        const auto key = std::make_tuple(r.scene, r.cam.width, r.cam.height);
        auto it = key_est.find(key);
        if (it != key_est.end()) return it->second.keys;
        int64_t k = 0;
        if (o.simulate) {
            k = (int64_t)((r.cam.width + 15) / 16) * ((r.cam.height + 15) / 16) * 64 +
                scenes[r.scene].scene.n / 8;
        } else {
            gs_job j = job_for(r);
            gs_ws_layout L;
            if (gs_forward_layout(&j, 1, 0, 0, &L) != GS_OK) return -1;
            size_t off;
            if (!arena.alloc(L.total_bytes, &off))
                // -3: the probe alone outgrows what the resident scenes leave of the
                // budget, so it can never run; -2: retry when memory frees up
                return L.total_bytes > arena.size - scene_bytes ? -3 : -2;
            int64_t kk = 0;
            const int rc = gs_count_keys(&j, 1, base + off, L.total_bytes, &kk, probe_stream);
            arena.release(off, L.total_bytes);
            if (rc != GS_OK) return -1;
            k = kk;
        }
        ClassEst& e = key_est[key];
        e.keys = std::max<int64_t>(k, 1);
        e.ms = model_ms(e.keys, scenes[r.scene].scene.n);
        e.samples = 0;
        return e.keys;
    }

    // frame-time estimate of a request whose class has been probed
    double estimate_ms(const Req& r) {
        const auto it = key_est.find(std::make_tuple(r.scene, r.cam.width, r.cam.height));
        return it == key_est.end() ? 0.0 : it->second.ms;
    }

    bool is_heavy(const Req& r) { return o.heavy_ms > 0 && estimate_ms(r) >= o.heavy_ms; }

    void finish(Req& r, int status) {
        r.status = status;
        r.finished = true;
        r.t_done = now_s();
        r.slot = r.job = -1;
        if (status == GS_OK) ++st_completed; else ++st_failed;
        if (status != GS_OK && r.has_out) {
            arena.release(r.out_off, r.out_bytes);
            r.has_out = false;
        }
    }

    // A frame whose completion word holds its batch's sequence number is
    // complete (the compositing kernel released its outputs before the
    // store), even while the rest of its batch is still running.
    bool frame_done(const Req& r) {
        if (o.simulate || !o.work_queue || r.finished || r.slot < 0) return false;
        const Slot& s = slots[r.slot];
        return __atomic_load_n(&s.done_host[r.job], __ATOMIC_ACQUIRE) == s.seq;
    }

    void finish_from_flag(Req& r) {
        r.flag_done = true;
        ++st_flag_done;
        finish(r, GS_OK);
    }

    void reap(Slot& s) {
        for (uint64_t t : s.tickets) {
            auto it = reqs.find(t);
            if (it != reqs.end() && frame_done(it->second)) finish_from_flag(it->second);
        }
        bool fail = false, overflow = false;
        uint32_t needed = 0;
        float batch_ms = -1.f;
        if (o.simulate) {
            fail = s.sim_fail;
        } else {
            const hipError_t e = hipEventQuery(s.event);
            if (e == hipErrorNotReady) return;
            fail = (e != hipSuccess);
            if (!fail) {
                needed = s.counters_host[0];
                overflow = s.counters_host[1] != 0u;
                if (hipEventElapsedTime(&batch_ms, s.ev_start, s.event) != hipSuccess) batch_ms = -1.f;
            }
        }
        if (o.simulate && now_s() < s.sim_done_at) return;
        // a single frame's measured time refines its class estimate
        const auto first = s.tickets.size() == 1 ? reqs.find(s.tickets[0]) : reqs.end();
        if (!fail && !overflow && batch_ms > 0.f && first != reqs.end()) {
            const Req& r = first->second;
            ClassEst& e = key_est[std::make_tuple(r.scene, r.cam.width, r.cam.height)];
            e.ms = e.samples == 0 ? (double)batch_ms : 0.7 * e.ms + 0.3 * (double)batch_ms;
            ++e.samples;
        }
        arena.release(s.ws_off, s.ws_bytes);
        std::vector<uint64_t> retry;
        for (uint64_t t : s.tickets) {
            // (a frame finished from its completion word may already be released)
            auto it = reqs.find(t);
            if (it == reqs.end() || it->second.finished) continue;
            Req& r = it->second;
            if (fail) {
                finish(r, GS_ERR_HIP);
            } else if (overflow) {
                const auto key = std::make_tuple(r.scene, r.cam.width, r.cam.height);
                const double scale = (double)needed / (double)std::max<int64_t>(s.cap, 1);
                ClassEst& e = key_est[key];
                e.keys = std::max<int64_t>(e.keys, (int64_t)(r.cap * scale / o.key_factor) + 1);
                if (++r.retries > 2) {
                    finish(r, GS_ERR_CAPACITY);
                } else {
                    if (r.has_out) {
                        arena.release(r.out_off, r.out_bytes);
                        r.has_out = false;
                    }
                    retry.push_back(t);
                }
            } else {
                finish(r, GS_OK);
            }
        }
        for (auto it = retry.rbegin(); it != retry.rend(); ++it) pending.push_front(*it);
        s.busy = false;
        s.heavy = false;
        s.tickets.clear();
    }

    // Builds and launches one batch on slot s; returns false when nothing could start.
    bool launch(Slot& s) {
        std::vector<uint64_t> take;
        std::vector<gs_job> jobs;
        int64_t cap = 0;
        const int maxb = o.fifo ? 1 : o.max_batch;
        bool busy_any = false, heavy_busy = false;
        for (const Slot& q : slots) {
            busy_any = busy_any || q.busy;
            heavy_busy = heavy_busy || (q.busy && q.heavy);
        }
        bool heavy_batch = false;
        while (!pending.empty() && (int)take.size() < maxb) {
            Req& r = reqs[pending.front()];
            const int64_t est = estimate_keys(r);
            if (est == -2) break;
            if (est == -3) {
                pending.pop_front();
                finish(r, GS_ERR_TOO_LARGE);
                continue;
            }
            if (est < 0) {
                pending.pop_front();
                finish(r, GS_ERR_HIP);
                continue;
            }
            if (!o.fifo) {
                // a heavy frame starts alone, once the device is free, and ends
                // the batch; beside it only tiny frames start (a quarter of
                // the heavy threshold and below), which stretch it little and
                // would otherwise wait its whole length
                const bool tiny = o.heavy_ms > 0 && estimate_ms(r) <= 0.25 * o.heavy_ms;
                if (heavy_busy && !tiny) break;
                if (is_heavy(r)) {
                    if (!take.empty() || busy_any) break;
                    heavy_batch = true;
                }
            }
            r.cap = std::max<int64_t>(1, (int64_t)(est * o.key_factor * (1 << r.retries)));
            r.out_bytes = out_bytes_for(r.cam.width, r.cam.height);
            size_t off;
            if (!arena.alloc(r.out_bytes, &off)) break;
            r.out_off = off;
            r.has_out = true;
            r.out = o.simulate ? gs_outputs{} : outputs_at(off, r.cam.width, r.cam.height);
            // does the batch workspace still fit with this request in it?
            jobs.push_back(job_for(r));
            gs_ws_layout L;
            const int rc = gs_forward_layout(jobs.data(), (int)jobs.size(), cap + r.cap, 0, &L);
            size_t wso;
            const bool fits = rc == GS_OK && arena.alloc(L.total_bytes, &wso);
            if (fits) arena.release(wso, L.total_bytes);
            if (!fits) {
                jobs.pop_back();
                arena.release(r.out_off, r.out_bytes);
                r.has_out = false;
                if (take.empty() && rc == GS_OK &&
                    L.total_bytes + align256(r.out_bytes) > arena.size - scene_bytes) {
                    // even an otherwise empty arena could not hold it
                    pending.pop_front();
                    finish(r, GS_ERR_TOO_LARGE);
                    continue;
                }
                break;
            }
            cap += r.cap;
            take.push_back(pending.front());
            pending.pop_front();
            if (heavy_batch) break;
        }
        if (take.empty()) return false;
        // shortest frames first: the compositing queue completes the batch's
        // frames in job order
        if (!o.fifo && take.size() > 1) {
            std::vector<size_t> ord(take.size());
            for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
            std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
                return estimate_ms(reqs[take[a]]) < estimate_ms(reqs[take[b]]);
            });
            std::vector<uint64_t> t2;
            std::vector<gs_job> j2;
            for (size_t k : ord) {
                t2.push_back(take[k]);
                j2.push_back(jobs[k]);
            }
            take.swap(t2);
            jobs.swap(j2);
        }
        s.heavy = heavy_batch;
        gs_ws_layout L;
        gs_forward_layout(jobs.data(), (int)jobs.size(), cap, 0, &L);
        size_t wso = 0;
        arena.alloc(L.total_bytes, &wso);   // checked above
        s.ws_off = wso;
        s.ws_bytes = L.total_bytes;
        s.cap = cap;
        s.tickets = take;
        s.busy = true;
        const double t = now_s();
        s.seq = s.seq + 1u ? s.seq + 1u : 1u;
        const int slot_idx = (int)(&s - slots.data());
        for (size_t k = 0; k < take.size(); ++k) {
            Req& r = reqs[take[k]];
            r.t_start = t;
            r.batch_size = (int)take.size();
            r.slot = slot_idx;
            r.job = (int)k;
        }
        ++st_batches;
        st_maxbatch = std::max<int64_t>(st_maxbatch, (int64_t)take.size());
        ++batch_counter;
        if (o.simulate) {
            s.sim_done_at = t + 1e-6 * o.sim_batch_us;
            s.sim_fail = o.sim_fail_every > 0 && (batch_counter % o.sim_fail_every) == 0;
            return true;
        }
        int rc = hipEventRecord(s.ev_start, s.stream) == hipSuccess ? GS_OK : GS_ERR_HIP;
        if (rc == GS_OK)
            rc = o.work_queue ? gs::render_forward_signalled(jobs.data(), (int)jobs.size(), base + wso, L.total_bytes,
                                                             cap, s.done_dev, s.seq, s.stream)
                              : gs_render_forward_batch(jobs.data(), (int)jobs.size(), base + wso, L.total_bytes, cap,
                                                        s.stream);
        if (rc == GS_OK &&
            hipMemcpyAsync(s.counters_host, base + wso + L.counters, 16, hipMemcpyDeviceToHost, s.stream) != hipSuccess)
            rc = GS_ERR_HIP;
        if (rc == GS_OK && hipEventRecord(s.event, s.stream) != hipSuccess) rc = GS_ERR_HIP;
        if (rc != GS_OK) {
            (void)hipStreamSynchronize(s.stream);
            arena.release(s.ws_off, s.ws_bytes);
            for (uint64_t tk : take) finish(reqs[tk], rc);
            s.busy = false;
            s.tickets.clear();
        }
        return true;
    }

    void run() {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            bool any_busy = false;
            for (auto& s : slots)
                if (s.busy) reap(s);
            if (!stop) {
                for (auto& s : slots) {
                    if (s.busy) continue;
                    if (o.fifo) {
                        bool other = false;
                        for (auto& q : slots) other = other || q.busy;
                        if (other) break;
                    }
                    if (!launch(s)) break;
                }
            }
            for (auto& s : slots) any_busy = any_busy || s.busy;
            if (stop && !any_busy) break;
            if (any_busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                cv.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }
};

extern "C" {

int gs_server_create(const gs_server_opts* opts, gs_server** server) {
    if (!opts || !server) return set_error(GS_ERR_INVALID_ARG, "null argument");
    gs_server_opts o = *opts;
    if (o.max_batch < 1 || o.max_batch > GS_MAX_BATCH) return set_error(GS_ERR_INVALID_ARG, "max_batch out of range");
    if (o.queue_depth < 1) return set_error(GS_ERR_INVALID_ARG, "queue_depth must be >= 1");
    if (o.n_streams < 1 || o.n_streams > 8) return set_error(GS_ERR_INVALID_ARG, "n_streams not in 1..8");
    if (!(o.key_factor >= 1.0)) return set_error(GS_ERR_INVALID_ARG, "key_factor must be >= 1");
    if (!(o.heavy_ms >= 0.0)) return set_error(GS_ERR_INVALID_ARG, "heavy_ms must be >= 0");
    if (o.hbm_budget_bytes < (1u << 20)) return set_error(GS_ERR_INVALID_ARG, "budget below 1 MiB");
    gs_server* s = new gs_server();
    s->o = o;
    s->arena.init(o.hbm_budget_bytes);
    s->slots.resize(o.n_streams);
    if (o.simulate) {
        // bookkeeping-only addresses: never dereferenced, never passed to a kernel
        s->base = reinterpret_cast<char*>((uintptr_t)1 << 40);
    } else {
        if (hipMalloc((void**)&s->base, s->arena.size) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return set_error(GS_ERR_OOM, "cannot reserve %zu bytes of device memory", o.hbm_budget_bytes);
        }
        bool ok = hipStreamCreateWithFlags(&s->probe_stream, hipStreamNonBlocking) == hipSuccess;
        for (auto& sl : s->slots) {
            ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&sl.event, hipEventDefault) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&sl.ev_start, hipEventDefault) == hipSuccess;
            ok = ok && hipHostMalloc((void**)&sl.counters_host, 64, hipHostMallocDefault) == hipSuccess;
            ok = ok && hipHostMalloc((void**)&sl.done_host, GS_MAX_BATCH * sizeof(uint32_t), hipHostMallocCoherent) ==
                           hipSuccess;
            if (ok) {
                memset(sl.done_host, 0, GS_MAX_BATCH * sizeof(uint32_t));
                ok = hipHostGetDevicePointer((void**)&sl.done_dev, sl.done_host, 0) == hipSuccess;
            }
        }
        if (!ok) {
            gs_server_destroy(s);
            return set_error(GS_ERR_HIP, "stream / event / pinned buffer creation failed");
        }
    }
    s->worker = std::thread([s] { s->run(); });
    *server = s;
    return GS_OK;
}

int gs_server_destroy(gs_server* s) {
    if (!s) return set_error(GS_ERR_INVALID_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (!s->o.simulate) {
        for (auto& sl : s->slots) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
            if (sl.event) (void)hipEventDestroy(sl.event);
            if (sl.ev_start) (void)hipEventDestroy(sl.ev_start);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
            if (sl.counters_host) (void)hipHostFree(sl.counters_host);
            if (sl.done_host) (void)hipHostFree(sl.done_host);
        }
        if (s->probe_stream) (void)hipStreamDestroy(s->probe_stream);
        if (s->base) (void)hipFree(s->base);
    }
    s->base = nullptr;
    delete s;
    return GS_OK;
}

int gs_scene_register(gs_server* s, const gs_scene* scene, int32_t* scene_id) {
    if (!s || !scene || !scene_id) return set_error(GS_ERR_INVALID_ARG, "null argument");
    if (scene->n < 0 || scene->sh_degree < 0 || scene->sh_degree > GS_MAX_SH_DEGREE)
        return set_error(GS_ERR_INVALID_ARG, "invalid scene");
    const size_t n = (size_t)scene->n;
    const size_t K = (size_t)(scene->sh_degree + 1) * (scene->sh_degree + 1);
    const size_t sz[5] = {12 * n, 12 * n, 16 * n, 4 * n, 12 * K * n};
    size_t total = 0;
    for (size_t b : sz) total += align256(b);
    std::lock_guard<std::mutex> lk(s->mu);
    size_t off;
    if (!s->arena.alloc(total, &off))
        return set_error(GS_ERR_OOM, "scene of %zu bytes does not fit the remaining budget", total);
    SceneRec rec;
    rec.off = off;
    rec.bytes = total;
    rec.scene = *scene;
    const void* src[5] = {scene->means, scene->log_scales, scene->quats, scene->opacity_logits, scene->sh};
    const float** dst[5] = {&rec.scene.means, &rec.scene.log_scales, &rec.scene.quats, &rec.scene.opacity_logits,
                            &rec.scene.sh};
    size_t o = off;
    for (int k = 0; k < 5; ++k) {
        char* p = s->base + o;
        *dst[k] = (const float*)p;
        if (!s->o.simulate && sz[k]) {
            if (hipMemcpy(p, src[k], sz[k], hipMemcpyDeviceToDevice) != hipSuccess) {
                s->arena.release(off, total);
                return set_error(GS_ERR_HIP, "scene copy failed: %s", hipGetErrorString(hipGetLastError()));
            }
        }
        o += align256(sz[k]);
    }
    s->scenes.push_back(rec);
    s->scene_bytes += s->arena.size ? align256(total) : 0;
    *scene_id = (int32_t)s->scenes.size() - 1;
    return GS_OK;
}

int gs_submit(gs_server* s, int32_t scene_id, const gs_camera* cam, const gs_render_opts* opts, uint64_t* ticket) {
    if (!s || !cam || !opts || !ticket) return set_error(GS_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (scene_id < 0 || scene_id >= (int32_t)s->scenes.size()) {
        return set_error(GS_ERR_NOT_FOUND, "unknown scene %d", scene_id);
    }
    if ((int)s->pending.size() >= s->o.queue_depth) {
        ++s->st_rejected;
        return set_error(GS_ERR_AGAIN, "queue full (%d pending)", (int)s->pending.size());
    }
    Req r;
    r.scene = scene_id;
    r.cam = *cam;
    r.opts = *opts;
    gs_job j = s->job_for(r);
    j.out.final_T = (float*)256;
    j.out.n_contrib = (uint32_t*)256;
    gs_ws_layout L;
    const int rc = gs_forward_layout(&j, 1, 0, 0, &L);
    if (rc != GS_OK) {
        ++s->st_rejected;
        return rc;
    }
    if (L.total_bytes + out_bytes_for(cam->width, cam->height) > s->arena.size - s->scene_bytes) {
        ++s->st_rejected;
        return set_error(GS_ERR_TOO_LARGE, "request needs more than the budget the resident scenes leave");
    }
    r.ticket = s->next_ticket++;
    r.t_submit = now_s();
    s->reqs[r.ticket] = r;
    s->pending.push_back(r.ticket);
    ++s->st_submitted;
    *ticket = r.ticket;
    s->cv.notify_all();
    return GS_OK;
}

int gs_poll(gs_server* s, uint64_t ticket, gs_result* result) {
    if (!s || !result) return set_error(GS_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(GS_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Req& r = it->second;
    if (s->frame_done(r)) s->finish_from_flag(r);
    if (!r.finished) return GS_ERR_NOT_READY;
    memset(result, 0, sizeof(*result));
    result->status = r.status;
    result->width = r.cam.width;
    result->height = r.cam.height;
    result->batch_size = r.batch_size;
    result->retries = r.retries;
    result->flag_done = r.flag_done ? 1 : 0;
    if (r.status == GS_OK) result->out = r.out;
    result->t_submit = r.t_submit;
    result->t_start = r.t_start;
    result->t_done = r.t_done;
    return GS_OK;
}

int gs_release(gs_server* s, uint64_t ticket) {
    if (!s) return set_error(GS_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(GS_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.finished) return set_error(GS_ERR_NOT_READY, "request still in flight");
    if (it->second.has_out) s->arena.release(it->second.out_off, it->second.out_bytes);
    s->reqs.erase(it);
    s->cv.notify_all();
    return GS_OK;
}

int gs_server_stats(gs_server* s, int64_t* st) {
    if (!s || !st) return set_error(GS_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st[0] = s->st_submitted;
    st[1] = s->st_completed;
    st[2] = s->st_failed;
    st[3] = s->st_rejected;
    st[4] = s->st_batches;
    st[5] = s->st_maxbatch;
    st[6] = (int64_t)s->arena.used;
    st[7] = (int64_t)s->arena.peak;
    st[8] = s->st_flag_done;
    return GS_OK;
}

}  // extern "C"
