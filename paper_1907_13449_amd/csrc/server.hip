// Request loop with continuous batching.
//
// One scheduler thread owns the device side.  Each turn it
//   1. retires batches whose completion event has fired: their arena extent is
//      freed and their requests are marked done;
//   2. admits pending requests into a new batch when fewer than max_inflight
//      batches are on the device: in arrival order, a request joins if the
//      batch's workspace (every member's lf_depth workspace plus the plan's
//      launch tables) still fits in the largest free extent of the arena and,
//      with group_ratio, if its own workspace is of the first member's size
//      class; a request that does not join is passed over and keeps its place;
//   3. plans the batch over that extent, launches it on a free stream and
//      records an event after it.
// Batches launched on different streams overlap on the device, so requests
// that arrive while others run start as soon as memory and a stream are free.
// The arena is one device allocation owned by the caller; the server carves it
// and never allocates device memory.
#include "lf_internal.h"

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxInflight = 4;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

using Clock = std::chrono::steady_clock;

struct Pending {
    int64_t ticket;
    lf_request q;
    size_t bytes;             // its lf_depth workspace, aligned
    hipEvent_t ready;         // recorded on the submitter's stream
    bool ready_failed;        // it could not be recorded: the request fails with LF_EDEVICE
    lf_request_info info;
};

struct Batch {
    int64_t id;
    std::vector<Pending> reqs;
    size_t off = 0, len = 0;  // arena extent
    lf_plan* plan = nullptr;
    int slot = -1;            // stream / event index
    int large = 0;            // large requests among its members
};

}  // namespace

struct lf_server {
    lf_server_config cfg;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_sched;   // work for the scheduler
    std::condition_variable cv_done;    // a request finished
    bool stop = false;
    std::thread th;

    std::deque<Pending> pending;
    std::unordered_set<int64_t> live;   // submitted and not yet waited for
    std::unordered_map<int64_t, lf_request_info> done;
    int64_t next_ticket = 1;
    int64_t next_batch = 0;
    int64_t completed = 0;

    std::map<size_t, size_t> free_ext;  // offset -> length
    size_t in_use = 0, peak = 0;

    std::vector<Batch> inflight;
    int large_inflight = 0;             // large requests of the batches on the device
    hipStream_t streams[kMaxInflight] = {};
    hipEvent_t events[kMaxInflight] = {};
    bool slot_busy[kMaxInflight] = {};
    bool device_ready = false;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    // --- arena: first fit over a sorted free list, neighbours merged on free ---
    size_t largest_free() const {
        size_t m = 0;
        for (auto& e : free_ext) m = std::max(m, e.second);
        return m;
    }
    bool alloc(size_t len, size_t* off) {
        for (auto it = free_ext.begin(); it != free_ext.end(); ++it) {
            if (it->second < len) continue;
            *off = it->first;
            const size_t rest = it->second - len;
            const size_t at = it->first + len;
            free_ext.erase(it);
            if (rest) free_ext[at] = rest;
            in_use += len;
            peak = std::max(peak, in_use);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t len) {
        if (!len) return;
        in_use -= len;
        auto it = free_ext.emplace(off, len).first;
        auto next = std::next(it);
        if (next != free_ext.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_ext.erase(next);
        }
        if (it != free_ext.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_ext.erase(it);
            }
        }
    }

    // Events of finished requests, kept for reuse (guarded by mu).
    std::vector<hipEvent_t> event_pool;

    void finish(Pending& r, int32_t status) {
        if (r.ready) event_pool.push_back(r.ready);
        r.ready = nullptr;
        r.info.status = status;
        r.info.t_done = now();
        done[r.ticket] = r.info;
        ++completed;
    }

    hipError_t init_device() {
        if (device_ready) return hipSuccess;
        hipError_t e = hipSuccess;
        for (int i = 0; i < cfg.max_inflight && e == hipSuccess; ++i) {
            e = hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&events[i], hipEventDisableTiming);
        }
        if (e != hipSuccess) {                  // undo a partial set-up; retried next batch
            for (int i = 0; i < kMaxInflight; ++i) {
                if (events[i]) (void)hipEventDestroy(events[i]);
                if (streams[i]) (void)hipStreamDestroy(streams[i]);
                events[i] = nullptr;
                streams[i] = nullptr;
            }
            return e;
        }
        device_ready = true;
        return hipSuccess;
    }

    bool is_large(const Pending& r) const { return (int64_t)r.bytes > cfg.large_bytes; }

    // Picks the members of the next batch (called with the lock held).
    bool form_batch(Batch& b) {
        const size_t room = largest_free();
        size_t total = 0;
        std::vector<lf_request> qs;
        size_t head = 0;                          // workspace of the first member
        int large = large_inflight;
        for (auto it = pending.begin(); it != pending.end() && (int)qs.size() < cfg.max_batch;) {
            if (head && cfg.group_ratio >= 2 &&
                (it->bytes > head * (size_t)cfg.group_ratio ||
                 it->bytes * (size_t)cfg.group_ratio < head)) {
                ++it;                                 // another size class: a later batch
                continue;
            }
            if (is_large(*it) && large >= cfg.max_large) {
                ++it;                                 // waits for a large one to finish
                continue;
            }
            qs.push_back(it->q);
            const size_t need = lf_batch_workspace_size(qs.data(), (int)qs.size());
            if (need != 0 && need <= room) {
                total = need;
                if (!head) head = it->bytes;
                if (is_large(*it)) {
                    ++large;
                    ++b.large;
                }
                b.reqs.push_back(*it);
                it = pending.erase(it);
            } else {
                qs.pop_back();
                ++it;
            }
        }
        if (b.reqs.empty()) return false;
        // a batch of one runs lf_depth's launches directly: its own workspace only
        b.len = align_up(b.reqs.size() == 1 ? b.reqs[0].bytes : total);
        if (!alloc(b.len, &b.off)) {   // cannot happen: total <= the largest extent
            for (auto r = b.reqs.rbegin(); r != b.reqs.rend(); ++r) pending.push_front(*r);
            b.reqs.clear();
            return false;
        }
        large_inflight += b.large;
        b.id = next_batch++;
        const double t = now();
        for (Pending& r : b.reqs) {
            r.info.t_admit = t;
            r.info.batch = b.id;
            r.info.batch_size = (int32_t)b.reqs.size();
        }
        return true;
    }

    // Plans and launches a formed batch (without the lock).  Returns the status
    // every member gets if it failed.
    lf_status launch_batch(Batch& b) {
        if (hipError_t e = init_device(); e != hipSuccess)
            return lf::record_error(LF_EDEVICE, "server streams: %s", hipGetErrorString(e));
        std::vector<lf_request> qs;
        for (const Pending& r : b.reqs) qs.push_back(r.q);
        hipStream_t st = streams[b.slot];
        // each member's inputs were produced on its submitter's stream
        for (const Pending& r : b.reqs) {
            if (r.ready_failed || !r.ready)
                return lf::record_error(LF_EDEVICE, "%s",
                                        "a request's ordering event could not be recorded");
            if (hipError_t e = hipStreamWaitEvent(st, r.ready, 0); e != hipSuccess)
                return lf::record_error(LF_EDEVICE, "server stream wait: %s",
                                        hipGetErrorString(e));
        }
        void* ws = (char*)cfg.arena + b.off;
        lf_status s = LF_OK;
        if (b.reqs.size() == 1) {
            // one light field: its launches directly, no plan tables to build or upload
            const lf_request& q = b.reqs[0].q;
            if ((s = lf_depth(&q.views, q.hyp, q.N, &q.params, q.disparity, q.d_index, ws,
                              b.len, st)) != LF_OK)
                return s;
        } else {
            if ((s = lf_plan_create(qs.data(), (int)qs.size(), ws, b.len, &cfg.tuning, st,
                                    &b.plan)) != LF_OK)
                return s;
            if ((s = lf_plan_run(b.plan, st)) != LF_OK) return s;
        }
        if (hipError_t e = hipEventRecord(events[b.slot], st); e != hipSuccess)
            return lf::record_error(LF_EDEVICE, "server event: %s", hipGetErrorString(e));
        return LF_OK;
    }

    void retire(Batch& b, int32_t status) {
        large_inflight -= b.large;
        for (Pending& r : b.reqs) finish(r, status);
        if (b.plan) lf_plan_destroy(b.plan);
        b.plan = nullptr;
        release(b.off, b.len);
        if (b.slot >= 0) slot_busy[b.slot] = false;
    }

    void loop() {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            // 1. completed batches
            bool retired = false;
            for (size_t i = 0; i < inflight.size();) {
                const hipError_t q = hipEventQuery(events[inflight[i].slot]);
                if (q == hipErrorNotReady) {
                    ++i;
                    continue;
                }
                retire(inflight[i], q == hipSuccess ? LF_OK : LF_EDEVICE);
                inflight.erase(inflight.begin() + i);
                retired = true;
            }
            if (retired) cv_done.notify_all();
            // 2. shutdown: cancel what has not started, drain what has
            if (stop) {
                for (Pending& r : pending) finish(r, LF_ECANCELED);
                pending.clear();
                cv_done.notify_all();
                if (inflight.empty()) break;
            }
            // 3. admission
            while (!stop && !pending.empty() && (int)inflight.size() < cfg.max_inflight) {
                Batch b;
                if (!form_batch(b)) break;
                for (int s = 0; s < cfg.max_inflight; ++s)
                    if (!slot_busy[s]) {
                        b.slot = s;
                        break;
                    }
                slot_busy[b.slot] = true;
                lk.unlock();
                const lf_status s = launch_batch(b);
                lk.lock();
                if (s != LF_OK) {
                    // a batch that could not be enqueued completes at once with the error
                    if (b.plan || b.reqs.size() == 1) {
                        // work may have been enqueued before the failure: wait for the stream
                        lk.unlock();
                        (void)hipStreamSynchronize(streams[b.slot]);
                        lk.lock();
                    }
                    retire(b, s);
                    cv_done.notify_all();
                    continue;
                }
                const double t = now();
                for (Pending& r : b.reqs) r.info.t_launch = t;
                inflight.push_back(std::move(b));
            }
            // 4. idle: sleep until a submission or a stop.  Busy: poll the events
            //    again at once (a timed sleep would add its oversleep, tens of
            //    microseconds, to every request's latency).
            if (inflight.empty()) {
                cv_sched.wait(lk, [&] { return stop || !pending.empty(); });
            } else {
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            }
        }
    }
};

extern "C" {

lf_status lf_server_create(const lf_server_config* cfg, lf_server** out) {
    if (!out) return lf::record_error(LF_EINVAL, "%s", "output pointer is NULL");
    *out = nullptr;
    if (!cfg) return lf::record_error(LF_EINVAL, "%s", "config is NULL");
    if (!cfg->arena || (uintptr_t)cfg->arena % kAlign || cfg->arena_bytes < kAlign)
        return lf::record_error(LF_EINVAL, "%s", "arena NULL, unaligned or empty");
    if (cfg->max_batch < 1 || cfg->max_inflight < 1 || cfg->max_inflight > kMaxInflight ||
        cfg->max_queue < 1 || cfg->group_ratio < 0 || cfg->group_ratio == 1 ||
        cfg->large_bytes < 0 || cfg->max_large < 0 || cfg->max_large > kMaxInflight)
        return lf::record_error(LF_EINVAL, "%s",
                                "max_batch >= 1, 1 <= max_inflight <= 4, max_queue >= 1, "
                                "group_ratio 0 or >= 2, large_bytes >= 0, 0 <= max_large <= 4");
    lf_server* s = new lf_server();
    s->cfg = *cfg;
    if (s->cfg.large_bytes == 0) s->cfg.large_bytes = (int64_t)256 << 20;
    if (s->cfg.max_large == 0) s->cfg.max_large = 1;
    s->cfg.arena_bytes = cfg->arena_bytes / kAlign * kAlign;
    s->t0 = Clock::now();
    s->free_ext[0] = s->cfg.arena_bytes;
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return LF_OK;
}

lf_status lf_server_submit(lf_server* srv, const lf_request* req, hipStream_t stream,
                           int64_t* ticket) {
    if (!srv || !ticket) return lf::record_error(LF_EINVAL, "%s", "NULL argument");
    lf_status st = lf::validate_request(req, 0, nullptr);
    if (st != LF_OK) return st;
    const size_t alone = lf_batch_workspace_size(req, 1);
    if (alone == 0 || alone > srv->cfg.arena_bytes)
        return lf::record_error(LF_ENOSPACE, "%s", "request workspace exceeds the arena");
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->stop) return lf::record_error(LF_ECANCELED, "%s", "server is stopping");
    if ((int)srv->pending.size() >= srv->cfg.max_queue)
        return lf::record_error(LF_EBUSY, "%s", "request queue is full");
    Pending p{};
    // the ordering event; if it cannot be made or recorded the request is still
    // queued and completes with LF_EDEVICE, like any other device failure
    if (!srv->event_pool.empty()) {
        p.ready = srv->event_pool.back();
        srv->event_pool.pop_back();
    } else if (hipEventCreateWithFlags(&p.ready, hipEventDisableTiming) != hipSuccess) {
        p.ready = nullptr;
    }
    p.ready_failed = !p.ready || hipEventRecord(p.ready, stream) != hipSuccess;
    p.ticket = srv->next_ticket++;
    p.q = *req;
    p.bytes = align_up(lf::request_workspace_bytes(req));
    p.info.t_submit = srv->now();
    p.info.batch = -1;
    p.info.status = LF_OK;
    srv->pending.push_back(p);
    srv->live.insert(p.ticket);
    *ticket = p.ticket;
    srv->cv_sched.notify_one();
    return LF_OK;
}

lf_status lf_server_wait(lf_server* srv, int64_t ticket, double timeout_s, lf_request_info* info) {
    if (!srv) return lf::record_error(LF_EINVAL, "%s", "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (!srv->live.count(ticket)) return lf::record_error(LF_EINVAL, "%s", "unknown ticket");
    auto ready = [&] { return srv->done.count(ticket) != 0; };
    if (timeout_s < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        return lf::record_error(LF_ETIMEOUT, "%s", "request still running");
    }
    const lf_request_info r = srv->done[ticket];
    srv->done.erase(ticket);
    srv->live.erase(ticket);
    if (info) *info = r;
    if (r.status != LF_OK) return lf::record_error((lf_status)r.status, "%s", "request failed");
    return LF_OK;
}

void lf_server_stats(const lf_server* srv, int64_t* completed, int64_t* batches,
                     int64_t* arena_in_use, int64_t* arena_peak) {
    if (!srv) return;
    lf_server* s = const_cast<lf_server*>(srv);
    std::lock_guard<std::mutex> g(s->mu);
    if (completed) *completed = s->completed;
    if (batches) *batches = s->next_batch;
    if (arena_in_use) *arena_in_use = (int64_t)s->in_use;
    if (arena_peak) *arena_peak = (int64_t)s->peak;
}

void lf_server_destroy(lf_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
    }
    srv->cv_sched.notify_all();
    srv->th.join();
    for (hipEvent_t e : srv->event_pool) (void)hipEventDestroy(e);
    if (srv->device_ready)
        for (int i = 0; i < srv->cfg.max_inflight; ++i) {
            if (srv->events[i]) (void)hipEventDestroy(srv->events[i]);
            if (srv->streams[i]) (void)hipStreamDestroy(srv->streams[i]);
        }
    delete srv;
}

}  // extern "C"
