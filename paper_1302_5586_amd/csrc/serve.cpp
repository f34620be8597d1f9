// Filter server: continuous batching of filter requests under an HBM
// budget, on one GPU.
//
// Requests are independent filter calls, so any set of admitted requests
// can share one persistent batch launch (every output element is an
// independent iteration, Sec. II-B.3). The engine thread admits requests
// first-come first-served while their device bytes fit in the budget,
// packs admitted requests into a batch whenever one of its streams is idle
// and launches the batch kernel there; completions are observed through
// per-stream events. New arrivals therefore run while earlier batches are
// still on the device. Each request's variant and tile shape come from the
// tune table keyed by (kind, radius, pixels) only, so a result is the same
// whichever batch the request lands in.
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pf_internal.h"

namespace pf {
namespace {

int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

constexpr int64_t kAlign = 256;

// First-fit allocator over one device block, with coalescing of free runs.
class Arena {
   public:
    void reset(int64_t size) {
        free_.clear();
        if (size > 0) free_[0] = size;
        used_ = 0;
    }
    // Returns the offset, or -1 if no free run is large enough.
    int64_t alloc(int64_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest > 0) free_[off + bytes] = rest;
                used_ += bytes;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t used() const { return used_; }

   private:
    std::map<int64_t, int64_t> free_;
    int64_t used_ = 0;
};

enum State { kQueued = 0, kAdmitted = 1, kLaunched = 2, kDone = 3, kFailed = 4 };

struct Request {
    int64_t ticket = 0;
    int32_t h = 0, w = 0, r = 0, kind = 0, var = 0, by = 16;
    const float *in_dev = nullptr;  // resident input, or null when uploaded
    std::vector<float> in_host;     // upload mode: copy of the caller's image
    std::vector<float> filt;        // weights (host copy)
    int64_t in_off = -1, out_off = -1;
    int64_t bytes = 0;              // bytes reserved in the arena
    int64_t t_arrival = 0, t_done = 0;
    bool auto_release = false;
    State state = kQueued;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<std::shared_ptr<Request>> reqs;
    void *dev = nullptr;  // descriptors, weights and task table
    void *host = nullptr; // pinned staging for the same bytes
    size_t cap = 0;
};

}  // namespace
}  // namespace pf

using namespace pf;

struct pf_server {
    int64_t budget = 0;
    int32_t max_batch = 64, max_queue = 1 << 16, flags = 0;
    int device = 0;
    char *arena_dev = nullptr;
    Arena arena;
    std::vector<Slot> slots;

    std::mutex mu;                     // guards everything below
    std::condition_variable cv_work;   // engine wakes on submit / stop
    std::condition_variable cv_done;   // waiters wake on completion
    std::deque<std::shared_ptr<Request>> queued;
    std::deque<std::shared_ptr<Request>> admitted;
    std::unordered_map<int64_t, std::shared_ptr<Request>> tickets;
    int64_t next_ticket = 1;
    bool stop = false;
    pf_status dev_error = PF_OK;
    std::string dev_error_msg;

    // statistics
    int64_t submitted = 0, n_admitted = 0, completed = 0, rejected = 0, batches = 0, pixels = 0;
    int64_t batched_reqs = 0, bytes_hw = 0, queue_hw = 0;
    int64_t first_arrival = INT64_MAX, last_done = 0;
    std::vector<double> lat_us;

    std::thread engine;
};

namespace pf {
namespace {

int64_t request_bytes(int h, int w, bool upload) {
    const int64_t img = ((int64_t)h * w * 4 + kAlign - 1) / kAlign * kAlign;
    return upload ? 2 * img : img;
}

// Release a finished request's arena bytes (lock held).
void release_locked(pf_server *s, const std::shared_ptr<Request> &q) {
    if (q->out_off >= 0) s->arena.release(q->out_off, (int64_t)q->h * q->w * 4);
    if (q->in_off >= 0) s->arena.release(q->in_off, (int64_t)q->h * q->w * 4);
    q->out_off = q->in_off = -1;
    s->tickets.erase(q->ticket);
}

// Build and launch one batch on slot k (lock NOT held; the requests are
// owned by the slot). Returns a status; on failure nothing is in flight.
pf_status launch_slot(pf_server *s, Slot &sl) {
    const bool exact = (s->flags & PF_FLAG_EXACT) != 0;
    std::vector<BatchImg> imgs[2];
    int64_t ntiles[2] = {0, 0};
    std::vector<float> weights;
    int used[2] = {0, 0};
    for (auto &q : sl.reqs) {
        const int g = q->r <= 4 ? 0 : 1;
        BatchImg d;
        d.in_off = q->in_dev ? (int64_t)((uintptr_t)q->in_dev / 4) : (int64_t)(((uintptr_t)s->arena_dev + q->in_off) / 4);
        d.out_off = (int64_t)(((uintptr_t)s->arena_dev + q->out_off) / 4);
        d.filt_off = (int64_t)weights.size();
        weights.insert(weights.end(), q->filt.begin(), q->filt.end());
        d.h = q->h;
        d.w = q->w;
        d.r = q->r;
        d.var = q->var;
        d.by = q->by;
        used[g] |= 1 << q->var;
        ntiles[g] += set_strips(d);
        imgs[g].push_back(d);
    }
    const int wpg = 4;
    int mask[2], grid[2] = {0, 0};
    std::vector<BatchTask> tasks[2];
    for (int g = 0; g < 2; ++g) {
        mask[g] = batch_mask(g, used[g]);
        if (!ntiles[g]) continue;
        grid[g] = batch_grid(g, exact, mask[g], wpg, ntiles[g]);
        tasks[g].reserve((size_t)ntiles[g]);
        for (size_t i = 0; i < imgs[g].size(); ++i) append_tiles(tasks[g], (int32_t)i, imgs[g][i]);
    }
    // Layout: [weights][imgs0][imgs1][tasks0][tasks1], 256-byte aligned parts.
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off_w = 0, off_i[2], off_t[2], bytes = up(weights.size() * 4);
    for (int g = 0; g < 2; ++g) {
        off_i[g] = bytes;
        bytes = up(bytes + imgs[g].size() * sizeof(BatchImg));
    }
    for (int g = 0; g < 2; ++g) {
        off_t[g] = bytes;
        bytes = up(bytes + tasks[g].size() * sizeof(BatchTask));
    }
    hipError_t e;
    if (bytes > sl.cap) {
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        sl.dev = sl.host = nullptr;
        sl.cap = 0;
        const size_t cap = std::max<size_t>(bytes * 2, 1 << 20);
        if ((e = hipMalloc(&sl.dev, cap)) != hipSuccess) return fail_hip(e, "server slot buffer");
        if ((e = hipHostMalloc(&sl.host, cap, hipHostMallocDefault)) != hipSuccess) return fail_hip(e, "server staging");
        sl.cap = cap;
    }
    char *h = (char *)sl.host;
    memcpy(h + off_w, weights.data(), weights.size() * 4);
    for (int g = 0; g < 2; ++g) {
        memcpy(h + off_i[g], imgs[g].data(), imgs[g].size() * sizeof(BatchImg));
        memcpy(h + off_t[g], tasks[g].data(), tasks[g].size() * sizeof(BatchTask));
    }
    // Upload-mode inputs first, then descriptors, then the kernels.
    for (auto &q : sl.reqs)
        if (!q->in_dev) {
            e = hipMemcpyAsync(s->arena_dev + q->in_off, q->in_host.data(), (size_t)q->h * q->w * 4, hipMemcpyHostToDevice,
                               sl.stream);
            if (e != hipSuccess) return fail_hip(e, "server input upload");
        }
    if ((e = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, sl.stream)) != hipSuccess)
        return fail_hip(e, "server descriptor upload");
    for (int g = 0; g < 2; ++g) {
        if (!ntiles[g]) continue;
        e = launch_batch(g, exact, mask[g], (const BatchImg *)((char *)sl.dev + off_i[g]),
                         (const BatchTask *)((char *)sl.dev + off_t[g]), (int)ntiles[g], grid[g], wpg, nullptr,
                         (const float *)sl.dev, nullptr, sl.stream);
        if (e != hipSuccess) return fail_hip(e, "server batch launch");
    }
    if ((e = hipEventRecord(sl.done, sl.stream)) != hipSuccess) return fail_hip(e, "server event");
    return PF_OK;
}

void engine_main(pf_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progressed = false;
        // Admission: first come, first served, while the bytes fit.
        while (!s->queued.empty()) {
            auto &q = s->queued.front();
            const bool upload = q->in_dev == nullptr;
            const int64_t img = (int64_t)q->h * q->w * 4;
            const int64_t out_off = s->arena.alloc(img);
            if (out_off < 0) break;
            int64_t in_off = -1;
            if (upload) {
                in_off = s->arena.alloc(img);
                if (in_off < 0) {
                    s->arena.release(out_off, img);
                    break;
                }
            }
            q->out_off = out_off;
            q->in_off = in_off;
            q->state = kAdmitted;
            s->bytes_hw = std::max(s->bytes_hw, s->arena.used());
            ++s->n_admitted;
            s->admitted.push_back(q);
            s->queued.pop_front();
            progressed = true;
        }
        // Completions.
        const int64_t t = now_ns();
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            for (auto &r : sl.reqs) {
                r->t_done = t;
                if (q == hipSuccess) {
                    r->state = kDone;
                    ++s->completed;
                    s->pixels += (int64_t)r->h * r->w;
                    s->lat_us.push_back((double)(t - r->t_arrival) / 1000.0);
                    s->last_done = std::max(s->last_done, t);
                } else {
                    r->state = kFailed;
                    s->dev_error = PF_EDEVICE;
                    s->dev_error_msg = std::string("batch failed: ") + hipGetErrorName(q);
                }
                if (r->auto_release) release_locked(s, r);
            }
            sl.reqs.clear();
            sl.busy = false;
            progressed = true;
            s->cv_done.notify_all();
        }
        // Launch admitted requests on idle streams.
        for (Slot &sl : s->slots) {
            if (sl.busy || s->admitted.empty()) continue;
            const size_t n = std::min<size_t>(s->admitted.size(), (size_t)s->max_batch);
            for (size_t i = 0; i < n; ++i) {
                sl.reqs.push_back(s->admitted.front());
                s->admitted.pop_front();
            }
            for (auto &r : sl.reqs) r->state = kLaunched;
            sl.busy = true;
            lk.unlock();
            const pf_status st = launch_slot(s, sl);
            lk.lock();
            ++s->batches;
            s->batched_reqs += (int64_t)sl.reqs.size();
            if (st != PF_OK) {
                s->dev_error = st;
                s->dev_error_msg = pf_last_error();
                for (auto &r : sl.reqs) {
                    r->state = kFailed;
                    if (r->auto_release) release_locked(s, r);
                }
                sl.reqs.clear();
                sl.busy = false;
                s->cv_done.notify_all();
            }
            progressed = true;
        }
        bool inflight = false;
        for (Slot &sl : s->slots) inflight |= sl.busy;
        if (s->stop && s->queued.empty() && s->admitted.empty() && !inflight) break;
        if (progressed) continue;
        if (inflight) {
            // Poll for completions without holding the lock.
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
}

pf_status submit_locked(pf_server *s, std::shared_ptr<Request> q, int64_t *ticket) {
    if ((int64_t)s->queued.size() >= s->max_queue) {
        ++s->rejected;
        return fail(PF_EAGAIN, "server queue is full");
    }
    q->ticket = s->next_ticket++;
    s->tickets[q->ticket] = q;
    s->queued.push_back(q);
    ++s->submitted;
    s->first_arrival = std::min(s->first_arrival, q->t_arrival);
    s->queue_hw = std::max(s->queue_hw, (int64_t)s->queued.size());
    *ticket = q->ticket;
    s->cv_work.notify_one();
    return PF_OK;
}

pf_status make_request(pf_server *s, int32_t h, int32_t w, int32_t r, int32_t kind, const float *in, int32_t in_is_host,
                       const float *filt, int64_t arrival_ns, std::shared_ptr<Request> *out) {
    if (h < 1 || w < 1) return fail(PF_EINVAL, "image sizes must be >= 1");
    if (r < 0 || r > PF_R_MAX) return fail(PF_EINVAL, "radius outside 0.." + std::to_string(PF_R_MAX));
    if (r > PF_BATCH_R_MAX)
        return fail(PF_EUNSUPPORTED, "served requests take radii 0.." + std::to_string(PF_BATCH_R_MAX));
    if (kind != PF_KIND_2D && kind != PF_KIND_SEP) return fail(PF_EINVAL, "unknown filter kind");
    if (!in || !filt) return fail(PF_EINVAL, "null pointer");
    if (!in_is_host && (uintptr_t)in % 4) return fail(PF_EINVAL, "device input must be 4-byte aligned");
    if ((int64_t)h * w > INT32_MAX) return fail(PF_EUNSUPPORTED, "image larger than 2^31-1 elements");
    const int64_t need = request_bytes(h, w, in_is_host != 0);
    if (need > s->budget) ++s->rejected;
    if (need > s->budget) return fail(PF_EBUDGET, "request needs " + std::to_string(need) + " bytes, budget is " + std::to_string(s->budget));
    auto q = std::make_shared<Request>();
    q->h = h;
    q->w = w;
    q->r = r;
    q->kind = kind;
    const int k = 2 * r + 1;
    const int nf = kind == PF_KIND_2D ? k * k : 2 * k;
    q->filt.assign(filt, filt + nf);
    const pf_tune_entry e = tune_lookup_batch(kind, r, (int64_t)h * w);
    q->var = kind == PF_KIND_2D ? PF_VAR_DIRECT : (e.variant == PF_VAR_SEP_DIRECT ? PF_VAR_SEP_DIRECT : PF_VAR_SEPARABLE);
    q->by = e.rows_per_wave;
    if (in_is_host)
        q->in_host.assign(in, in + (size_t)h * w);
    else
        q->in_dev = in;
    q->bytes = need;
    q->t_arrival = arrival_ns ? arrival_ns : now_ns();
    *out = q;
    return PF_OK;
}

pf_status lookup(pf_server *s, int64_t ticket, std::shared_ptr<Request> *q) {
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(PF_EINVAL, "unknown or released ticket " + std::to_string(ticket));
    *q = it->second;
    return PF_OK;
}

double percentile(std::vector<double> &v, double p) {
    if (v.empty()) return 0.0;
    const size_t i = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + i, v.end());
    return v[i];
}

}  // namespace
}  // namespace pf

extern "C" {

pf_status pf_server_create(int64_t hbm_budget_bytes, int32_t n_streams, int32_t max_batch, int32_t max_queue,
                           int32_t flags, pf_server **const __restrict srv) {
    clear_error();
    if (!srv) return fail(PF_EINVAL, "null server out-parameter");
    *srv = nullptr;
    if (hbm_budget_bytes < kAlign) return fail(PF_EINVAL, "budget must be at least 256 bytes");
    if (n_streams < 1 || n_streams > 8) return fail(PF_EINVAL, "n_streams outside 1..8");
    if (max_batch < 1 || max_batch > 4096) return fail(PF_EINVAL, "max_batch outside 1..4096");
    if (max_queue < 1) return fail(PF_EINVAL, "max_queue must be >= 1");
    if (flags & ~PF_FLAG_EXACT) return fail(PF_EINVAL, "unknown flags");
    auto *s = new (std::nothrow) pf_server;
    if (!s) return fail(PF_ENOMEM, "server allocation");
    s->budget = hbm_budget_bytes;
    s->max_batch = max_batch;
    s->max_queue = max_queue;
    s->flags = flags;
    (void)hipGetDevice(&s->device);
    hipError_t e = hipMalloc(&s->arena_dev, (size_t)hbm_budget_bytes);
    if (e != hipSuccess) {
        delete s;
        return fail_hip(e, "server arena");
    }
    s->arena.reset(hbm_budget_bytes);
    s->slots.resize(n_streams);
    for (Slot &sl : s->slots) {
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess) {
            pf_status st = fail_hip(e, "server streams");
            for (Slot &x : s->slots) {
                if (x.done) (void)hipEventDestroy(x.done);
                if (x.stream) (void)hipStreamDestroy(x.stream);
            }
            (void)hipFree(s->arena_dev);
            delete s;
            return st;
        }
    }
    s->engine = std::thread(engine_main, s);
    *srv = s;
    return PF_OK;
}

pf_status pf_server_submit(pf_server *s, int32_t h, int32_t w, int32_t r, int32_t kind, const float *in,
                           int32_t in_is_host, const float *filt, int64_t arrival_ns, int64_t *const __restrict ticket) {
    clear_error();
    if (!s || !ticket) return fail(PF_EINVAL, "null argument");
    std::shared_ptr<Request> q;
    pf_status st;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(PF_EINVAL, "server is shutting down");
        st = make_request(s, h, w, r, kind, in, in_is_host, filt, arrival_ns, &q);
        if (st) return st;
        return submit_locked(s, q, ticket);
    }
}

pf_status pf_server_poll(pf_server *s, int64_t ticket, int32_t *const __restrict done) {
    clear_error();
    if (!s || !done) return fail(PF_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::shared_ptr<Request> q;
    if (pf_status st = lookup(s, ticket, &q)) return st;
    if (q->state == kFailed) return fail(PF_EDEVICE, s->dev_error_msg);
    *done = q->state == kDone;
    return PF_OK;
}

pf_status pf_server_wait(pf_server *s, int64_t ticket, int64_t timeout_ns) {
    clear_error();
    if (!s) return fail(PF_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    std::shared_ptr<Request> q;
    if (pf_status st = lookup(s, ticket, &q)) return st;
    auto ready = [&] { return q->state == kDone || q->state == kFailed; };
    if (timeout_ns < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready)) {
        return fail(PF_ETIMEDOUT, "request " + std::to_string(ticket) + " not done");
    }
    if (q->state == kFailed) return fail(PF_EDEVICE, s->dev_error_msg);
    return PF_OK;
}

pf_status pf_server_result(pf_server *s, int64_t ticket, int32_t h, int32_t w, float *out, int32_t out_is_host) {
    clear_error();
    if (!s || !out) return fail(PF_EINVAL, "null argument");
    std::shared_ptr<Request> q;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (pf_status st = lookup(s, ticket, &q)) return st;
        if (q->state == kFailed) return fail(PF_EDEVICE, s->dev_error_msg);
        if (q->state != kDone) return fail(PF_EAGAIN, "request not done");
        if (h != q->h || w != q->w) return fail(PF_EINVAL, "size differs from the request's");
    }
    const hipError_t e = hipMemcpy(out, s->arena_dev + q->out_off, (size_t)h * w * 4,
                                   out_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice);
    std::lock_guard<std::mutex> lk(s->mu);
    release_locked(s, q);
    s->cv_work.notify_one();
    if (e != hipSuccess) return fail_hip(e, "result copy");
    return PF_OK;
}

pf_status pf_server_release(pf_server *s, int64_t ticket) {
    clear_error();
    if (!s) return fail(PF_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    std::shared_ptr<Request> q;
    if (pf_status st = lookup(s, ticket, &q)) return st;
    if (q->state != kDone && q->state != kFailed) return fail(PF_EAGAIN, "request not done");
    release_locked(s, q);
    s->cv_work.notify_one();
    return PF_OK;
}

pf_status pf_server_stats_get(pf_server *s, pf_server_stats *const __restrict st) {
    clear_error();
    if (!s || !st) return fail(PF_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(st, 0, sizeof *st);
    st->submitted = s->submitted;
    st->admitted = s->n_admitted;
    st->completed = s->completed;
    st->rejected = s->rejected;
    st->batches = s->batches;
    st->pixels = s->pixels;
    st->bytes_high_water = s->bytes_hw;
    st->queue_high_water = s->queue_hw;
    st->mean_batch = s->batches ? (double)s->batched_reqs / (double)s->batches : 0.0;
    std::vector<double> v = s->lat_us;
    st->p50_us = percentile(v, 0.50);
    st->p99_us = percentile(v, 0.99);
    st->p999_us = percentile(v, 0.999);
    st->max_us = v.empty() ? 0.0 : *std::max_element(v.begin(), v.end());
    if (s->completed && s->last_done > s->first_arrival) {
        st->wall_s = (double)(s->last_done - s->first_arrival) * 1e-9;
        st->gpx_per_s = (double)s->pixels / st->wall_s * 1e-9;
    }
    return PF_OK;
}

pf_status pf_server_run_trace(pf_server *s, int32_t n, const int64_t *__restrict arrival_ns, const int32_t *__restrict h,
                              const int32_t *__restrict w, const int32_t *__restrict r,
                              const int64_t *__restrict pix_off, const int64_t *__restrict filt_off, int64_t npix,
                              const float *in, int64_t nfilt, const float *filt) {
    clear_error();
    if (!s || n < 1 || !arrival_ns || !h || !w || !r || !pix_off || !filt_off || !in || !filt)
        return fail(PF_EINVAL, "bad trace arguments");
    for (int i = 0; i < n; ++i) {
        const int64_t px = (int64_t)h[i] * w[i];
        if (h[i] < 1 || w[i] < 1 || pix_off[i] < 0 || pix_off[i] > npix - px)
            return fail(PF_EINVAL, "trace request " + std::to_string(i) + " outside the pool");
        if (r[i] < 0 || r[i] > PF_R_MAX || filt_off[i] < 0 || filt_off[i] > nfilt - 2 * (2 * r[i] + 1))
            return fail(PF_EINVAL, "trace request " + std::to_string(i) + " has a bad filter");
        if (i && arrival_ns[i] < arrival_ns[i - 1]) return fail(PF_EINVAL, "arrival times must not decrease");
    }
    const int64_t t0 = now_ns();
    int64_t last_ticket = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t due = t0 + arrival_ns[i];
        // Open loop: sleep until shortly before the scheduled time, then spin.
        for (;;) {
            const int64_t left = due - now_ns();
            if (left <= 0) break;
            if (left > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(left - 100000));
            else std::this_thread::yield();
        }
        std::shared_ptr<Request> q;
        std::lock_guard<std::mutex> lk(s->mu);
        pf_status st = make_request(s, h[i], w[i], r[i], PF_KIND_SEP, in + pix_off[i], 0, filt + filt_off[i], due, &q);
        if (st) return st;
        q->auto_release = true;
        int64_t t;
        if ((st = submit_locked(s, q, &t))) return st;
        last_ticket = t;
    }
    (void)last_ticket;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->completed + (s->dev_error != PF_OK) >= s->submitted || s->dev_error != PF_OK; });
    if (s->dev_error != PF_OK) return fail(s->dev_error, s->dev_error_msg);
    return PF_OK;
}

pf_status pf_server_destroy(pf_server *s) {
    clear_error();
    if (!s) return PF_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->engine.joinable()) s->engine.join();
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
    }
    (void)hipFree(s->arena_dev);
    delete s;
    return PF_OK;
}

}  // extern "C"
