// Filter server: continuous batching of filter and reduction requests under
// an HBM budget, on one GPU.
//
// Requests are independent calls, so any set of admitted requests can share
// one batch of launches (every output element is an independent iteration,
// Sec. II-B.3; the sum and the histogram are the paper's reductions,
// Sec. II-B.3 and Sec. III-B). The engine thread admits requests first-come
// first-served while their device bytes fit in the budget, packs admitted
// requests into a batch whenever one of its streams is idle and launches
// there: the persistent filter kernel for the filter requests, then the
// multi-array sum and histogram kernels. Completions are observed through
// per-stream events, so new arrivals run while earlier batches are still on
// the device. Each filter request's variant and tile shape come from the
// tune table keyed by (kind, radius, pixels) only, and each reduction is
// computed part by part with the same device code as the single-array
// calls, so a result is the same whichever batch the request lands in.
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
constexpr int kOpFilter = 0;  // request kinds besides PF_OP_SUM_F32, PF_OP_HIST_U8
// Per-stream buffers allocated when the server is created (grown only for a
// batch that does not fit): descriptors and weights, and the reduction
// workspace.
constexpr size_t kSlotBytes = 1 << 20;
constexpr size_t kSlotWorkspace = 4 << 20;
// While other batches are on the device, a launch waits up to this long
// (from the oldest admitted request's arrival) for at least half a batch:
// under load, batches fill instead of leaving with whatever arrived since
// the last completion; with nothing in flight, a request launches at once.
constexpr int64_t kHoldNs = 50000;

int64_t round_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

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
        bytes = round_up(bytes);
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
        bytes = round_up(bytes);
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
    int32_t op = kOpFilter;
    int32_t h = 0, w = 0, r = 0, kind = 0, var = 0, by = 16;  // filter requests
    int64_t n = 0;                                             // reductions: elements
    const void *in_dev = nullptr;   // resident input, or null when uploaded
    std::vector<uint8_t> in_host;   // upload mode: copy of the caller's input
    std::vector<float> filt;        // weights (host copy)
    hipEvent_t ready = nullptr;     // recorded on the stream that produces in_dev
    int64_t in_off = -1, out_off = -1;
    int64_t in_bytes = 0, out_bytes = 0;
    int64_t t_arrival = 0, t_done = 0;
    bool auto_release = false;
    State state = kQueued;
    pf_status fail_status = PF_OK;
    std::string fail_msg;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<std::shared_ptr<Request>> reqs;
    void *dev = nullptr;   // descriptors, weights and task tables
    void *host = nullptr;  // pinned staging for the same bytes
    size_t cap = 0;
    void *ws = nullptr;    // reduction workspace: chunk partials, span sub-histograms
    size_t ws_cap = 0;
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
    // Bumped (under `mu`) whenever the engine has new work: a submit, a
    // release that frees arena bytes, shutdown. While batches are in flight
    // the engine takes the lock only when this moved or an event completed.
    std::atomic<int64_t> work_seq{0};
    std::condition_variable cv_done;   // waiters wake on completion
    std::deque<std::shared_ptr<Request>> queued;
    std::deque<std::shared_ptr<Request>> admitted;
    std::unordered_map<int64_t, std::shared_ptr<Request>> tickets;
    std::vector<hipEvent_t> events;    // free events for producer-stream ordering
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

// Release a finished request's arena bytes and ticket (lock held).
// Tell the engine that it has new work (the caller holds s->mu).
void wake_engine_locked(pf_server *s) {
    s->work_seq.fetch_add(1, std::memory_order_release);
    s->cv_work.notify_one();
}

void release_locked(pf_server *s, const std::shared_ptr<Request> &q) {
    if (q->out_off >= 0) s->arena.release(q->out_off, q->out_bytes);
    if (q->in_off >= 0) s->arena.release(q->in_off, q->in_bytes);
    q->out_off = q->in_off = -1;
    s->tickets.erase(q->ticket);
}

// Return a request's ordering event to the pool (lock held).
void drop_event_locked(pf_server *s, const std::shared_ptr<Request> &q) {
    if (q->ready) s->events.push_back(q->ready);
    q->ready = nullptr;
}

void fail_locked(pf_server *s, const std::shared_ptr<Request> &q, pf_status st, const std::string &msg) {
    q->state = kFailed;
    q->fail_status = st;
    q->fail_msg = msg;
    drop_event_locked(s, q);
    if (q->auto_release) release_locked(s, q);
}

// Grow a slot's staging (descriptors) or workspace buffer to `need` bytes.
pf_status ensure_slot(Slot &sl, size_t need, size_t need_ws) {
    hipError_t e;
    if (need > sl.cap) {
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        sl.dev = sl.host = nullptr;
        sl.cap = 0;
        const size_t cap = std::max<size_t>(need * 2, kSlotBytes);
        if ((e = hipMalloc(&sl.dev, cap)) != hipSuccess) return fail_hip(e, "server slot buffer");
        if ((e = hipHostMalloc(&sl.host, cap, hipHostMallocDefault)) != hipSuccess) return fail_hip(e, "server staging");
        sl.cap = cap;
    }
    if (need_ws > sl.ws_cap) {
        if (sl.ws) (void)hipFree(sl.ws);
        sl.ws = nullptr;
        sl.ws_cap = 0;
        const size_t cap = std::max<size_t>(need_ws * 2, kSlotWorkspace);
        if ((e = hipMalloc(&sl.ws, cap)) != hipSuccess) return fail_hip(e, "server reduction workspace");
        sl.ws_cap = cap;
    }
    return PF_OK;
}

// Build and launch one batch on a slot (lock NOT held; the requests are
// owned by the slot). Returns a status; on failure nothing is in flight.
pf_status launch_slot(pf_server *s, Slot &sl) {
    const bool exact = (s->flags & PF_FLAG_EXACT) != 0;
    auto arena_addr = [&](int64_t off) { return (int64_t)((uintptr_t)s->arena_dev + off); };
    // Filter requests: descriptors for the persistent batch kernel.
    std::vector<BatchImg> imgs;
    int64_t ntiles = 0;
    std::vector<float> weights;
    int used = 0;
    // Reduction requests: descriptors and part lists.
    std::vector<ReduceReq> rreqs;
    std::vector<int32_t> sum_ids, hist_ids;
    std::vector<ReduceTask> sum_tasks, hist_tasks;
    int64_t sum_parts = 0, hist_parts = 0;
    for (auto &q : sl.reqs) {
        const int64_t in_addr = q->in_dev ? (int64_t)(uintptr_t)q->in_dev : arena_addr(q->in_off);
        if (q->op == kOpFilter) {
            BatchImg d;
            d.in_off = in_addr / 4;
            d.out_off = arena_addr(q->out_off) / 4;
            d.filt_off = (int64_t)weights.size();
            weights.insert(weights.end(), q->filt.begin(), q->filt.end());
            d.h = q->h;
            d.w = q->w;
            d.r = q->r;
            d.var = q->var;
            d.by = q->by;
            used |= 1 << q->var;
            ntiles += set_strips(d);
            imgs.push_back(d);
        } else {
            ReduceReq d;
            d.in = in_addr;
            d.n = q->n;
            d.out = arena_addr(q->out_off);
            d.op = q->op;
            d.pad = 0;
            const int32_t id = (int32_t)rreqs.size();
            const int64_t parts = reduce_parts(q->op, q->n);
            if (q->op == PF_OP_SUM_F32) {
                d.first = sum_parts;
                sum_ids.push_back(id);
                for (int64_t p = 0; p < parts; ++p) sum_tasks.push_back({id, (int32_t)p});
                sum_parts += parts;
            } else {
                d.first = hist_parts;
                hist_ids.push_back(id);
                for (int64_t p = 0; p < parts; ++p) hist_tasks.push_back({id, (int32_t)p});
                hist_parts += parts;
            }
            rreqs.push_back(d);
        }
    }
    const int wpg = 4;
    int mask = 1, grid = 0;
    std::vector<BatchTask> tasks;
    if (ntiles) {
        if (ntiles > INT32_MAX || sum_tasks.size() > INT32_MAX || hist_tasks.size() > INT32_MAX)
            return fail(PF_EUNSUPPORTED, "batch too large");
        mask = batch_mask(0, used);
        grid = batch_grid(0, exact, mask, wpg, ntiles);
        tasks.reserve((size_t)ntiles);
        for (size_t i = 0; i < imgs.size(); ++i) append_tiles(tasks, (int32_t)i, imgs[i]);
    }
    // Layout: [weights][imgs][tasks][reduce reqs][sum ids][hist ids][sum tasks][hist tasks],
    // 256-byte aligned parts.
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    auto place = [&](size_t bytes) {
        const size_t o = off;
        off = up(off + bytes);
        return o;
    };
    const size_t o_w = place(weights.size() * 4);
    const size_t o_i = place(imgs.size() * sizeof(BatchImg));
    const size_t o_t = place(tasks.size() * sizeof(BatchTask));
    const size_t o_rq = place(rreqs.size() * sizeof(ReduceReq));
    const size_t o_si = place(sum_ids.size() * 4);
    const size_t o_hi = place(hist_ids.size() * 4);
    const size_t o_st = place(sum_tasks.size() * sizeof(ReduceTask));
    const size_t o_ht = place(hist_tasks.size() * sizeof(ReduceTask));
    const size_t bytes = off;
    const size_t ws_sum = up((size_t)sum_parts * sizeof(double));
    const size_t ws_bytes = ws_sum + (size_t)hist_parts * 256 * sizeof(uint32_t);
    if (pf_status st = ensure_slot(sl, bytes, ws_bytes)) return st;
    char *h = (char *)sl.host;
    auto put = [&](size_t o, const void *p, size_t n) {
        if (n) memcpy(h + o, p, n);
    };
    put(o_w, weights.data(), weights.size() * 4);
    put(o_i, imgs.data(), imgs.size() * sizeof(BatchImg));
    put(o_t, tasks.data(), tasks.size() * sizeof(BatchTask));
    put(o_rq, rreqs.data(), rreqs.size() * sizeof(ReduceReq));
    put(o_si, sum_ids.data(), sum_ids.size() * 4);
    put(o_hi, hist_ids.data(), hist_ids.size() * 4);
    put(o_st, sum_tasks.data(), sum_tasks.size() * sizeof(ReduceTask));
    put(o_ht, hist_tasks.data(), hist_tasks.size() * sizeof(ReduceTask));
    hipError_t e;
    // Device inputs: wait for the work their producer stream had queued at
    // submit. Upload-mode inputs: copy them into the arena.
    for (auto &q : sl.reqs) {
        if (q->ready) {
            if ((e = hipStreamWaitEvent(sl.stream, q->ready, 0)) != hipSuccess)
                return fail_hip(e, "server wait on the producer stream");
        } else if (!q->in_dev) {
            e = hipMemcpyAsync(s->arena_dev + q->in_off, q->in_host.data(), (size_t)q->in_bytes, hipMemcpyHostToDevice,
                               sl.stream);
            if (e != hipSuccess) return fail_hip(e, "server input upload");
        }
    }
    if ((e = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, sl.stream)) != hipSuccess)
        return fail_hip(e, "server descriptor upload");
    char *d = (char *)sl.dev;
    if (ntiles) {
        e = launch_batch(0, exact, mask, (const BatchImg *)(d + o_i), (const BatchTask *)(d + o_t), (int)ntiles, grid,
                         wpg, nullptr, (const float *)(d + o_w), nullptr, sl.stream);
        if (e != hipSuccess) return fail_hip(e, "server batch launch");
    }
    if (!rreqs.empty()) {
        e = launch_reduce_batch((const ReduceReq *)(d + o_rq), (const int32_t *)(d + o_si), (int)sum_ids.size(),
                                (const ReduceTask *)(d + o_st), (int)sum_tasks.size(), (const int32_t *)(d + o_hi),
                                (int)hist_ids.size(), (const ReduceTask *)(d + o_ht), (int)hist_tasks.size(),
                                (double *)sl.ws, (uint32_t *)((char *)sl.ws + ws_sum), sl.stream);
        if (e != hipSuccess) return fail_hip(e, "server reduction launch");
    }
    if ((e = hipEventRecord(sl.done, sl.stream)) != hipSuccess) return fail_hip(e, "server event");
    return PF_OK;
}

void engine_main(pf_server *s) {
    (void)hipSetDevice(s->device);
    // Only this thread touches the slots once it runs, so their events are
    // polled without the lock, and while batches run the lock is taken only
    // when there is something to do: a submitter at a high request rate then
    // finds it free instead of contending with a polling loop.
    std::vector<hipError_t> polled(s->slots.size(), hipErrorNotReady);
    std::unique_lock<std::mutex> lk(s->mu, std::defer_lock);
    int64_t seen = -1;       // work_seq when the lock was last taken
    int64_t hold_until = 0;  // a held launch is due by then (0: none)
    bool again = true;       // the last pass changed state: look again
    for (;;) {
        bool busy = false, finished = false;
        for (size_t i = 0; i < s->slots.size(); ++i) {
            polled[i] = hipErrorNotReady;
            if (!s->slots[i].busy) continue;
            busy = true;
            polled[i] = hipEventQuery(s->slots[i].done);
            finished |= polled[i] != hipErrorNotReady;
        }
        if (busy && !finished && !again && s->work_seq.load(std::memory_order_acquire) == seen &&
            (hold_until == 0 || now_ns() < hold_until)) {
            std::this_thread::yield();
            continue;
        }
        lk.lock();
        seen = s->work_seq.load(std::memory_order_relaxed);
        bool progressed = false;
        if (s->stop && !s->queued.empty()) {
            // Shutting down: requests not yet admitted fail (they may never
            // fit while finished, unreleased results hold the arena).
            for (auto &q : s->queued) fail_locked(s, q, PF_EAGAIN, "server shut down before the request was admitted");
            s->queued.clear();
            s->cv_done.notify_all();
        }
        // Admission: first come, first served, while the bytes fit.
        while (!s->queued.empty()) {
            auto &q = s->queued.front();
            const bool upload = q->in_dev == nullptr;
            const int64_t out_off = s->arena.alloc(q->out_bytes);
            if (out_off < 0) break;
            int64_t in_off = -1;
            if (upload) {
                in_off = s->arena.alloc(q->in_bytes);
                if (in_off < 0) {
                    s->arena.release(out_off, q->out_bytes);
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
        for (size_t i = 0; i < s->slots.size(); ++i) {
            Slot &sl = s->slots[i];
            const hipError_t q = polled[i];
            if (!sl.busy || q == hipErrorNotReady) continue;
            for (auto &r : sl.reqs) {
                r->t_done = t;
                drop_event_locked(s, r);
                if (q == hipSuccess) {
                    r->state = kDone;
                    ++s->completed;
                    if (r->op == kOpFilter) s->pixels += (int64_t)r->h * r->w;
                    s->lat_us.push_back((double)(t - r->t_arrival) / 1000.0);
                    s->last_done = std::max(s->last_done, t);
                    if (r->auto_release) release_locked(s, r);
                } else {
                    s->dev_error = PF_EDEVICE;
                    s->dev_error_msg = std::string("batch failed: ") + hipGetErrorName(q);
                    fail_locked(s, r, PF_EDEVICE, s->dev_error_msg);
                }
            }
            sl.reqs.clear();
            sl.busy = false;
            progressed = true;
            s->cv_done.notify_all();
        }
        // Launch admitted requests on idle streams.
        bool any_busy = false;
        for (Slot &sl : s->slots) any_busy |= sl.busy;
        const bool hold = any_busy && !s->stop && !s->admitted.empty() &&
                          (int64_t)s->admitted.size() < std::max(1, s->max_batch / 2) &&
                          now_ns() - s->admitted.front()->t_arrival < kHoldNs;
        hold_until = hold ? s->admitted.front()->t_arrival + kHoldNs : 0;
        for (Slot &sl : s->slots) {
            if (hold) break;
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
                // Work already enqueued on the stream (before the failing
                // call) must finish before the requests' memory is reused.
                (void)hipStreamSynchronize(sl.stream);
                for (auto &r : sl.reqs) fail_locked(s, r, st, s->dev_error_msg);
                sl.reqs.clear();
                sl.busy = false;
                s->cv_done.notify_all();
            }
            progressed = true;
        }
        bool inflight = false;
        for (Slot &sl : s->slots) inflight |= sl.busy;
        if (s->stop && s->queued.empty() && s->admitted.empty() && !inflight) break;
        if (!progressed && !inflight) s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
        lk.unlock();
        again = progressed || !inflight;
        if (!progressed && inflight) std::this_thread::yield();
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
    wake_engine_locked(s);
    return PF_OK;
}

// Bytes a request holds in the arena: its result, and its input when uploaded.
pf_status check_budget(pf_server *s, const Request &q, bool upload) {
    const int64_t need = round_up(q.out_bytes) + (upload ? round_up(q.in_bytes) : 0);
    if (need > s->budget) {
        ++s->rejected;
        return fail(PF_EBUDGET, "request needs " + std::to_string(need) + " bytes, budget is " + std::to_string(s->budget));
    }
    return PF_OK;
}

// Common part of a submit (lock held): copies an uploaded input, or orders a
// device input after the work queued on `stream` (order = false: the input
// is known to be complete).
pf_status stage_input(pf_server *s, Request &q, const void *in, bool upload, void *stream, bool order) {
    if (upload) {
        const uint8_t *b = (const uint8_t *)in;
        q.in_host.assign(b, b + q.in_bytes);
        return PF_OK;
    }
    q.in_dev = in;
    if (!order) return PF_OK;
    hipEvent_t ev = nullptr;
    if (!s->events.empty()) {
        ev = s->events.back();
        s->events.pop_back();
    } else {
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return fail_hip(e, "server ordering event");
    }
    hipError_t e = hipEventRecord(ev, (hipStream_t)stream);
    if (e != hipSuccess) {
        s->events.push_back(ev);
        return fail_hip(e, "server ordering event record");
    }
    q.ready = ev;
    return PF_OK;
}

pf_status make_request(pf_server *s, int32_t h, int32_t w, int32_t r, int32_t kind, const float *in, int32_t in_is_host,
                       const float *filt, void *stream, bool order, int64_t arrival_ns,
                       std::shared_ptr<Request> *out) {
    if (h < 1 || w < 1) return fail(PF_EINVAL, "image sizes must be >= 1");
    if (r < 0 || r > PF_R_MAX) return fail(PF_EINVAL, "radius outside 0.." + std::to_string(PF_R_MAX));
    if (r > PF_BATCH_R_MAX)
        return fail(PF_EUNSUPPORTED, "served requests take radii 0.." + std::to_string(PF_BATCH_R_MAX));
    if (kind != PF_KIND_2D && kind != PF_KIND_SEP) return fail(PF_EINVAL, "unknown filter kind");
    if (!in || !filt) return fail(PF_EINVAL, "null pointer");
    if (!in_is_host && (uintptr_t)in % 4) return fail(PF_EINVAL, "device input must be 4-byte aligned");
    if ((int64_t)h * w > INT32_MAX) return fail(PF_EUNSUPPORTED, "image larger than 2^31-1 elements");
    auto q = std::make_shared<Request>();
    q->op = kOpFilter;
    q->h = h;
    q->w = w;
    q->r = r;
    q->kind = kind;
    q->in_bytes = q->out_bytes = (int64_t)h * w * 4;
    if (pf_status st = check_budget(s, *q, in_is_host != 0)) return st;
    const int k = 2 * r + 1;
    const int nf = kind == PF_KIND_2D ? k * k : 2 * k;
    q->filt.assign(filt, filt + nf);
    const pf_tune_entry e = tune_lookup_batch(kind, r, (int64_t)h * w);
    q->var = kind == PF_KIND_2D ? PF_VAR_DIRECT : PF_VAR_SEPARABLE;
    q->by = e.rows_per_wave;
    if (pf_status st = stage_input(s, *q, in, in_is_host != 0, stream, order)) return st;
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

pf_status failed(const Request &q) { return fail(q.fail_status ? q.fail_status : PF_EDEVICE, q.fail_msg); }

double percentile(std::vector<double> &v, double p) {
    if (v.empty()) return 0.0;
    const size_t i = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + i, v.end());
    return v[i];
}

// Copy a finished request's result out and release it.
pf_status copy_result(pf_server *s, int64_t ticket, int32_t op, int32_t h, int32_t w, void *out, int32_t out_is_host) {
    if (!s || !out) return fail(PF_EINVAL, "null argument");
    std::shared_ptr<Request> q;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (pf_status st = lookup(s, ticket, &q)) return st;
        if (q->state == kFailed) return failed(*q);
        if (q->state != kDone) return fail(PF_EAGAIN, "request not done");
        if (q->op != op) return fail(PF_EINVAL, "the request is of another kind");
        if (op == kOpFilter && (h != q->h || w != q->w)) return fail(PF_EINVAL, "size differs from the request's");
    }
    const hipError_t e = hipMemcpy(out, s->arena_dev + q->out_off, (size_t)q->out_bytes,
                                   out_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice);
    std::lock_guard<std::mutex> lk(s->mu);
    release_locked(s, q);
    wake_engine_locked(s);
    if (e != hipSuccess) return fail_hip(e, "result copy");
    return PF_OK;
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
    auto cleanup = [&](pf_status st) {
        for (Slot &x : s->slots) {
            if (x.done) (void)hipEventDestroy(x.done);
            if (x.stream) (void)hipStreamDestroy(x.stream);
            if (x.dev) (void)hipFree(x.dev);
            if (x.host) (void)hipHostFree(x.host);
            if (x.ws) (void)hipFree(x.ws);
        }
        if (s->arena_dev) (void)hipFree(s->arena_dev);
        delete s;
        return st;
    };
    hipError_t e = hipMalloc(&s->arena_dev, (size_t)hbm_budget_bytes);
    if (e != hipSuccess) {
        s->arena_dev = nullptr;
        return cleanup(fail_hip(e, "server arena"));
    }
    s->arena.reset(hbm_budget_bytes);
    s->slots.resize(n_streams);
    for (Slot &sl : s->slots) {
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
            return cleanup(fail_hip(e, "server streams"));
        // Buffers sized for typical batches up front: no allocation (and its
        // device-wide synchronisation) on the serving path in steady state.
        if (pf_status st = ensure_slot(sl, kSlotBytes, kSlotWorkspace)) return cleanup(st);
    }
    s->engine = std::thread(engine_main, s);
    *srv = s;
    return PF_OK;
}

pf_status pf_server_submit(pf_server *s, int32_t h, int32_t w, int32_t r, int32_t kind, const float *in,
                           int32_t in_is_host, const float *filt, void *stream, int64_t arrival_ns,
                           int64_t *const __restrict ticket) {
    clear_error();
    if (!s || !ticket) return fail(PF_EINVAL, "null argument");
    std::shared_ptr<Request> q;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(PF_EINVAL, "server is shutting down");
    if (pf_status st = make_request(s, h, w, r, kind, in, in_is_host, filt, stream, true, arrival_ns, &q)) return st;
    if (pf_status st = submit_locked(s, q, ticket)) {
        drop_event_locked(s, q);
        return st;
    }
    return PF_OK;
}

pf_status pf_server_submit_reduce(pf_server *s, int32_t op, int64_t n, const void *in, int32_t in_is_host,
                                  void *stream, int64_t arrival_ns, int64_t *const __restrict ticket) {
    clear_error();
    if (!s || !ticket || !in) return fail(PF_EINVAL, "null argument");
    if (op != PF_OP_SUM_F32 && op != PF_OP_HIST_U8) return fail(PF_EINVAL, "unknown reduction");
    if (n < 1 || n > ((int64_t)1 << 40)) return fail(PF_EINVAL, "n must be in 1..2^40");
    if (op == PF_OP_SUM_F32 && !in_is_host && (uintptr_t)in % 4) return fail(PF_EINVAL, "x must be 4-byte aligned");
    if (reduce_parts(op, n) > INT32_MAX) return fail(PF_EUNSUPPORTED, "array too long");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(PF_EINVAL, "server is shutting down");
    auto q = std::make_shared<Request>();
    q->op = op;
    q->n = n;
    q->in_bytes = op == PF_OP_SUM_F32 ? n * 4 : n;
    q->out_bytes = op == PF_OP_SUM_F32 ? 2 * (int64_t)sizeof(double) : 256 * (int64_t)sizeof(int64_t);
    if (pf_status st = check_budget(s, *q, in_is_host != 0)) return st;
    if (pf_status st = stage_input(s, *q, in, in_is_host != 0, stream, true)) return st;
    q->t_arrival = arrival_ns ? arrival_ns : now_ns();
    if (pf_status st = submit_locked(s, q, ticket)) {
        drop_event_locked(s, q);
        return st;
    }
    return PF_OK;
}

pf_status pf_server_poll(pf_server *s, int64_t ticket, int32_t *const __restrict done) {
    clear_error();
    if (!s || !done) return fail(PF_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::shared_ptr<Request> q;
    if (pf_status st = lookup(s, ticket, &q)) return st;
    if (q->state == kFailed) return failed(*q);
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
    if (q->state == kFailed) return failed(*q);
    return PF_OK;
}

pf_status pf_server_result(pf_server *s, int64_t ticket, int32_t h, int32_t w, float *out, int32_t out_is_host) {
    clear_error();
    return copy_result(s, ticket, kOpFilter, h, w, out, out_is_host);
}

pf_status pf_server_result_reduce(pf_server *s, int64_t ticket, int32_t op, void *out, int32_t out_is_host) {
    clear_error();
    if (op != PF_OP_SUM_F32 && op != PF_OP_HIST_U8) return fail(PF_EINVAL, "unknown reduction");
    return copy_result(s, ticket, op, 0, 0, out, out_is_host);
}

pf_status pf_server_release(pf_server *s, int64_t ticket) {
    clear_error();
    if (!s) return fail(PF_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    std::shared_ptr<Request> q;
    if (pf_status st = lookup(s, ticket, &q)) return st;
    if (q->state != kDone && q->state != kFailed) return fail(PF_EAGAIN, "request not done");
    release_locked(s, q);
    wake_engine_locked(s);
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
    for (int i = 0; i < n;) {
        // Open loop: sleep until shortly before the next scheduled time, then
        // spin.
        for (;;) {
            const int64_t left = t0 + arrival_ns[i] - now_ns();
            if (left <= 0) break;
            if (left > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(left - 100000));
            else std::this_thread::yield();
        }
        // Everything already due goes in under one lock, each request with
        // its own scheduled arrival time: one lock hand-off per group instead
        // of per request when arrivals come faster than a submit.
        const int64_t now = now_ns();
        std::lock_guard<std::mutex> lk(s->mu);
        for (int g = 0; i < n && g < 256 && t0 + arrival_ns[i] <= now; ++i, ++g) {
            std::shared_ptr<Request> q;
            // The pool is complete before the call (documented): no ordering
            // event.
            pf_status st = make_request(s, h[i], w[i], r[i], PF_KIND_SEP, in + pix_off[i], 0, filt + filt_off[i],
                                        nullptr, false, t0 + arrival_ns[i], &q);
            if (st) return st;
            q->auto_release = true;
            int64_t t;
            if ((st = submit_locked(s, q, &t))) return st;
        }
    }
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->completed + (s->dev_error != PF_OK) >= s->submitted || s->dev_error != PF_OK; });
    if (s->dev_error != PF_OK) return fail(s->dev_error, s->dev_error_msg);
    return PF_OK;
}

pf_status pf_arena_replay(int64_t budget, int32_t n, const int64_t *__restrict op, int64_t *__restrict result,
                          int64_t *const __restrict used) {
    clear_error();
    if (budget < kAlign || n < 0 || (n > 0 && (!op || !result)) || !used) return fail(PF_EINVAL, "bad arguments");
    Arena a;
    a.reset(budget);
    std::vector<int64_t> live(n, -1);  // offset of live allocation i, or -1
    for (int32_t i = 0; i < n; ++i) {
        if (op[i] > 0) {
            result[i] = a.alloc(op[i]);
            live[i] = result[i];
        } else {
            const int64_t j = -op[i] - 1;
            if (j < 0 || j >= i || live[j] < 0) return fail(PF_EINVAL, "operation " + std::to_string(i) + " frees nothing");
            a.release(live[j], op[j]);
            live[j] = -1;
            result[i] = 0;
        }
    }
    *used = a.used();
    return PF_OK;
}

pf_status pf_server_destroy(pf_server *s) {
    clear_error();
    if (!s) return PF_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        wake_engine_locked(s);
    }
    if (s->engine.joinable()) s->engine.join();
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.ws) (void)hipFree(sl.ws);
    }
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    for (auto &kv : s->tickets)
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    (void)hipFree(s->arena_dev);
    delete s;
    return PF_OK;
}

}  // extern "C"
