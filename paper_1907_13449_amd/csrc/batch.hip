// Batch plans: many light fields per launch.
//
// A plan lays the light fields' workspaces out one after another in the
// caller's workspace, followed by the device tables of its grouped launches
// (one argument record per light field and launch, and the prefix sums of their
// block counts).  Recording runs the same stage functions as lf_depth with a
// recorder in place of a stream, so each stage becomes one launch per kernel
// variant over every light field of the batch.  The launches can be captured
// into a HIP graph and replayed with one graph launch.
//
// The autotuner times the schedule candidates on the plan's own light fields,
// stage by stage with HIP events, and keeps the fastest per stage.  Every
// candidate computes the same results.
#include "lf_internal.h"

#include <algorithm>
#include <cstring>
#include <memory>
#include <utility>

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMaxLaunches = 64;       // grouped launches per run (checked)

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t table_bytes(int n) {
    return kMaxLaunches * (align_up((size_t)n * lf::kMaxArgRecord) + align_up((size_t)(n + 1) * 4));
}

lf::Tuning to_tuning(const lf_tuning* t) {
    lf::Tuning u;
    if (!t) return u;
    if (t->cost_cells_per_thread) u.cost_cpt = t->cost_cells_per_thread;
    if (t->cost_stride) u.cost_stride = t->cost_stride;
    if (t->dense_prefetch) u.dense_depth = t->dense_prefetch;
    if (t->bounded_prefetch) u.bounded_depth = t->bounded_prefetch;
    if (t->bounded_lanes) u.bounded_lanes = t->bounded_lanes;
    if (t->bounded_offsets) u.bounded_offsets = t->bounded_offsets;
    return u;
}

lf_tuning from_tuning(const lf::Tuning& u) {
    return lf_tuning{u.cost_cpt,      u.cost_stride,   u.dense_depth,
                     u.bounded_depth, u.bounded_lanes, u.bounded_offsets};
}

bool valid_tuning(const lf::Tuning& u) {
    auto in = [](int v, std::initializer_list<int> ok) {
        return std::find(ok.begin(), ok.end(), v) != ok.end();
    };
    return in(u.cost_cpt, {2, 4, 8}) && in(u.cost_stride, {1, 2, 4}) &&
           in(u.dense_depth, {4, 8, 16}) && in(u.bounded_depth, {4, 8, 16}) &&
           in(u.bounded_lanes, {16, 32, 64}) && in(u.bounded_offsets, {32, 64});
}

}  // namespace

struct lf_plan : lf::Recorder {
    std::vector<lf_request> reqs;
    std::vector<lf::Job> jobs;
    lf::Tuning tune;
    char* dev_tables = nullptr;
    size_t table_cap = 0;
    std::vector<char> host_tables;
    std::vector<std::pair<int, std::function<hipError_t(hipStream_t)>>> launches;
    bool overflow = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    const void* table(const void* host, size_t bytes) override {
        const size_t at = align_up(host_tables.size());
        if (bytes > lf::kMaxArgRecord * jobs.size() + 4 || at + bytes > table_cap) {
            overflow = true;
            return dev_tables;
        }
        host_tables.resize(at + bytes);
        std::memcpy(host_tables.data() + at, host, bytes);
        return dev_tables + at;
    }
    void add(int stage, std::function<hipError_t(hipStream_t)> fn) override {
        launches.emplace_back(stage, std::move(fn));
    }

    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }

    // Records the launches under `t` and enqueues the table upload.
    lf_status record(const lf::Tuning& t, hipStream_t stream) {
        drop_graph();
        launches.clear();
        host_tables.clear();
        overflow = false;
        tune = t;
        lf::Runner r;
        r.rec = this;
        r.tune = t;
        lf::Jobs js;
        for (const lf::Job& j : jobs) js.push_back(&j);
        lf_status s = lf::run_depth_jobs(r, js);
        if (s != LF_OK) return s;
        if (overflow || launches.size() > kMaxLaunches)
            return lf::record_error(LF_EUNSUPPORTED, "%s", "batch plan tables overflow");
        if (!host_tables.empty()) {
            hipError_t e = hipMemcpyAsync(dev_tables, host_tables.data(), host_tables.size(),
                                          hipMemcpyHostToDevice, stream);
            if (e != hipSuccess)
                return lf::record_error(LF_EDEVICE, "plan table upload: %s", hipGetErrorString(e));
        }
        return LF_OK;
    }

    lf_status run(hipStream_t stream) {
        if (exec) {
            hipError_t e = hipGraphLaunch(exec, stream);
            if (e != hipSuccess)
                return lf::record_error(LF_EDEVICE, "graph launch: %s", hipGetErrorString(e));
            return LF_OK;
        }
        for (auto& l : launches) {
            hipError_t e = l.second(stream);
            if (e != hipSuccess)
                return lf::record_error(LF_EDEVICE, "batch launch: %s", hipGetErrorString(e));
        }
        return LF_OK;
    }

    // Runs once eagerly with an event at every stage boundary; adds each stage's
    // milliseconds to ms[].
    lf_status timed_run(hipStream_t stream, std::vector<hipEvent_t>& ev, double* ms) {
        std::vector<int> stage_of;
        int cur = -1;
        size_t k = 0;
        auto mark = [&](int st) -> hipError_t {
            if (k >= ev.size()) {
                hipEvent_t e;
                hipError_t x = hipEventCreate(&e);
                if (x != hipSuccess) return x;
                ev.push_back(e);
            }
            stage_of.push_back(st);
            return hipEventRecord(ev[k++], stream);
        };
        for (auto& l : launches) {
            if (l.first != cur) {
                if (hipError_t e = mark(l.first); e != hipSuccess)
                    return lf::record_error(LF_EDEVICE, "event: %s", hipGetErrorString(e));
                cur = l.first;
            }
            if (hipError_t e = l.second(stream); e != hipSuccess)
                return lf::record_error(LF_EDEVICE, "batch launch: %s", hipGetErrorString(e));
        }
        if (hipError_t e = mark(-1); e != hipSuccess)
            return lf::record_error(LF_EDEVICE, "event: %s", hipGetErrorString(e));
        if (hipError_t e = hipEventSynchronize(ev[k - 1]); e != hipSuccess)
            return lf::record_error(LF_EDEVICE, "event: %s", hipGetErrorString(e));
        for (size_t i = 0; i + 1 < k; ++i) {
            float t = 0.0f;
            (void)hipEventElapsedTime(&t, ev[i], ev[i + 1]);
            ms[stage_of[i]] += t;
        }
        return LF_OK;
    }
};

extern "C" {

size_t lf_batch_workspace_size(const lf_request* reqs, int32_t n) {
    if (!reqs || n < 1) return 0;
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (lf::validate_request(&reqs[i], 0, nullptr) != LF_OK) return 0;
        const size_t b = lf::request_workspace_bytes(&reqs[i]);
        if (b == 0) return 0;
        total += align_up(b);
    }
    return total + table_bytes(n);
}

lf_status lf_plan_create(const lf_request* reqs, int32_t n, void* ws, size_t ws_bytes,
                         const lf_tuning* tuning, hipStream_t stream, lf_plan** out) {
    if (!out) return lf::record_error(LF_EINVAL, "%s", "plan output pointer is NULL");
    *out = nullptr;
    if (!reqs || n < 1) return lf::record_error(LF_EINVAL, "%s", "empty batch");
    if (!ws || (uintptr_t)ws % kAlign)
        return lf::record_error(LF_EINVAL, "%s", "workspace NULL or not 256-byte aligned");
    const lf::Tuning t = to_tuning(tuning);
    if (!valid_tuning(t)) return lf::record_error(LF_EINVAL, "%s", "tuning value out of range");
    for (int i = 0; i < n; ++i) {
        lf_status s = lf::validate_request(&reqs[i], 0, nullptr);
        if (s != LF_OK) return s;
    }
    const size_t need = lf_batch_workspace_size(reqs, n);
    if (need == 0 || ws_bytes < need)
        return lf::record_error(LF_ENOSPACE, "%s", "batch workspace too small");
    std::unique_ptr<lf_plan> p(new lf_plan());
    p->reqs.assign(reqs, reqs + n);
    char* at = (char*)ws;
    for (int i = 0; i < n; ++i) {
        const size_t b = align_up(lf::request_workspace_bytes(&reqs[i]));
        p->jobs.push_back(lf::request_job(&reqs[i], at));
        at += b;
    }
    p->dev_tables = at;
    p->table_cap = table_bytes(n);
    lf_status s = p->record(t, stream);
    if (s != LF_OK) return s;
    *out = p.release();
    return LF_OK;
}

lf_status lf_plan_autotune(lf_plan* p, hipStream_t stream, int32_t reps, lf_tuning* chosen) {
    if (!p) return lf::record_error(LF_EINVAL, "%s", "plan is NULL");
    if (reps < 1) reps = 1;
    std::vector<hipEvent_t> ev;
    auto measure = [&](const lf::Tuning& t, double* ms) -> lf_status {
        for (int i = 0; i < lf::kNumStages; ++i) ms[i] = 0.0;
        lf_status s = p->record(t, stream);
        if (s != LF_OK) return s;
        double warm[lf::kNumStages] = {};
        if ((s = p->timed_run(stream, ev, warm)) != LF_OK) return s;   // warm-up
        for (int r = 0; r < reps; ++r)
            if ((s = p->timed_run(stream, ev, ms)) != LF_OK) return s;
        return LF_OK;
    };
    // Phase 1: candidate i takes the i-th value of every list; the stages are
    // timed separately, so each stage's parameter is chosen on its own.
    const int cpt[3] = {2, 4, 8}, dd[3] = {4, 8, 16}, bl[3] = {16, 32, 64};
    double best_cost = 1e30, best_dense = 1e30, best_bounded = 1e30;
    lf::Tuning best = p->tune;
    best.cost_stride = 1;
    best.bounded_depth = lf::Tuning{}.bounded_depth;   // the depth phase 1 runs at
    lf_status s = LF_OK;
    for (int i = 0; i < 3 && s == LF_OK; ++i) {
        lf::Tuning t;
        t.cost_cpt = cpt[i];
        t.cost_stride = 1;
        t.dense_depth = dd[i];
        t.bounded_lanes = bl[i];
        double ms[lf::kNumStages];
        if ((s = measure(t, ms)) != LF_OK) break;
        if (ms[lf::kStCost] < best_cost) best_cost = ms[lf::kStCost], best.cost_cpt = cpt[i];
        if (ms[lf::kStInitPaths] < best_dense)
            best_dense = ms[lf::kStInitPaths], best.dense_depth = dd[i];
        if (ms[lf::kStSgmFinal] < best_bounded)
            best_bounded = ms[lf::kStSgmFinal], best.bounded_lanes = bl[i];
    }
    // Phase 2: workgroups walking several cost slices, at the chosen slice size.
    for (int stride : {2, 4}) {
        if (s != LF_OK) break;
        lf::Tuning t = best;
        t.cost_stride = stride;
        double ms[lf::kNumStages];
        if ((s = measure(t, ms)) != LF_OK) break;
        if (ms[lf::kStCost] < best_cost) best_cost = ms[lf::kStCost], best.cost_stride = stride;
    }
    // Phase 3: the other prefetch depths of the bounded SGM with one line per wave.
    const int depth0 = best.bounded_depth;
    for (int depth : {4, 8, 16}) {
        if (s != LF_OK || best.bounded_lanes != 64) break;
        if (depth == depth0) continue;
        lf::Tuning t = best;
        t.bounded_depth = depth;
        double ms[lf::kNumStages];
        if ((s = measure(t, ms)) != LF_OK) break;
        if (ms[lf::kStSgmFinal] < best_bounded)
            best_bounded = ms[lf::kStSgmFinal], best.bounded_depth = depth;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (s != LF_OK) return s;
    if ((s = p->record(best, stream)) != LF_OK) return s;
    if (chosen) *chosen = from_tuning(best);
    return LF_OK;
}

lf_status lf_plan_capture(lf_plan* p) {
    if (!p) return lf::record_error(LF_EINVAL, "%s", "plan is NULL");
    if (p->exec) return LF_OK;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return lf::record_error(LF_EDEVICE, "stream: %s", hipGetErrorString(e));
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (auto& l : p->launches) {
            e = l.second(cs);
            if (e != hipSuccess) break;
        }
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) {
            p->graph = g;
            e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        p->drop_graph();
        return lf::record_error(LF_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    return LF_OK;
}

lf_status lf_plan_run(lf_plan* p, hipStream_t stream) {
    if (!p) return lf::record_error(LF_EINVAL, "%s", "plan is NULL");
    return p->run(stream);
}

int32_t lf_plan_launches(const lf_plan* p) { return p ? (int32_t)p->launches.size() : 0; }

lf_status lf_plan_tuning(const lf_plan* p, lf_tuning* out) {
    if (!p || !out) return lf::record_error(LF_EINVAL, "%s", "NULL argument");
    *out = from_tuning(p->tune);
    return LF_OK;
}

void lf_plan_destroy(lf_plan* p) {
    if (!p) return;
    p->drop_graph();
    delete p;
}

}  // extern "C"
