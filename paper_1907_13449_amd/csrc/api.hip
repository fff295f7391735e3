// Host side of liblf: argument validation, workspace planning and the order of
// launches for each C-ABI entry point declared in include/lf.h.
#include "lf_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

namespace lf {

int cross_views(int S, int T, int* st) {
    const int sh = (S - 1) / 2, th = (T - 1) / 2;
    const int cand[4][2] = {{sh, 0}, {sh, T - 1}, {0, th}, {S - 1, th}};
    int n = 0;
    for (int i = 0; i < 4; ++i) {
        const int s = cand[i][0], t = cand[i][1];
        if (s == sh && t == th) continue;
        bool dup = false;
        for (int j = 0; j < n; ++j) dup |= st[2 * j] == s && st[2 * j + 1] == t;
        if (dup) continue;
        st[2 * n] = s;
        st[2 * n + 1] = t;
        ++n;
    }
    return n;
}

}  // namespace lf

namespace {

thread_local std::string g_err;

lf_status fail(lf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

lf_status device_status(hipError_t e, const char* where) {
    if (e == hipSuccess) return LF_OK;
    return fail(LF_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define LF_CHECK(expr)                                  \
    do {                                                \
        lf_status _s = (expr);                          \
        if (_s != LF_OK) return _s;                     \
    } while (0)

#define LF_HIP(expr, where)                             \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return device_status(_e, where); \
    } while (0)

// Opt-in stage timing: a HIP event pair recorded on the call's stream around
// each group of launches.  Off by default; when off nothing is recorded.
namespace prof {
const char* const kNames[lf::kNumStages] = {
    "census",      "initial_cost", "initial_paths", "initial_sum_wta", "fuse_fill_borders",
    "offsets",     "cost_inputs",  "cost_bounded",  "sgm_bounded",     "wta_subpixel_median"};
struct Rec {
    int stage, launches;
    hipEvent_t a, b;
};
std::mutex mu;
bool on = false;
std::vector<Rec> pending;
std::vector<hipEvent_t> pool;

hipEvent_t get_event() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets the launches a runner issues while the scope lives.
struct Scope {
    int stage, before;
    const lf::Runner& r;
    hipEvent_t a = nullptr;
    Scope(int stage_, const lf::Runner& r_) : stage(stage_), before(r_.launches), r(r_) {
        std::lock_guard<std::mutex> g(mu);
        if (!on || r.rec) return;               // recorded launches are timed by their plan
        a = get_event();
        if (a && hipEventRecord(a, r.stream) != hipSuccess) {
            pool.push_back(a);
            a = nullptr;
        }
    }
    ~Scope() {
        if (!a) return;
        std::lock_guard<std::mutex> g(mu);
        hipEvent_t b = get_event();
        if (b && hipEventRecord(b, r.stream) == hipSuccess) {
            pending.push_back(Rec{stage, r.launches - before, a, b});
        } else {
            pool.push_back(a);
            if (b) pool.push_back(b);
        }
    }
};
}  // namespace prof

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's workspace: sizes first (base == nullptr),
// then the same sequence of take() calls hands out the pointers.
struct Carve {
    char* base;
    size_t used = 0;
    explicit Carve(void* b) : base((char*)b) {}
    void* take(size_t bytes) {
        void* p = base ? base + used : nullptr;
        used += align_up(bytes);
        return p;
    }
};

lf_status check_shape(int S, int T, int H, int W, int N) {
    if (S < 1 || T < 1 || S % 2 == 0 || T % 2 == 0)
        return fail(LF_EINVAL, "angular grid %dx%d: S and T must be odd and >= 1", S, T);
    if (S * T < 2) return fail(LF_EINVAL, "a light field needs at least 2 views");
    if (S > 65535 || T > 65535)
        return fail(LF_EUNSUPPORTED, "angular grid %dx%d (at most 65535 per side)", S, T);
    if (H < 1 || W < 1) return fail(LF_EINVAL, "image size %dx%d", H, W);
    if ((int64_t)H * W > (1 << 30) || H > LF_MAX_SIDE || W > LF_MAX_SIDE)
        return fail(LF_EUNSUPPORTED, "image of %d x %d pixels", H, W);
    if (N < 2) return fail(LF_EINVAL, "N = %d hypotheses (need >= 2)", N);
    if (N > LF_MAX_HYPOTHESES)
        return fail(LF_EUNSUPPORTED, "N = %d hypotheses (max %d)", N, LF_MAX_HYPOTHESES);
    return LF_OK;
}

lf_status check_views(const lf_view_set* v) {
    if (!v) return fail(LF_EINVAL, "views is NULL");
    if (!v->data) return fail(LF_EINVAL, "views->data is NULL");
    if (v->dtype != LF_U8 && v->dtype != LF_F32) return fail(LF_EINVAL, "dtype %d", v->dtype);
    if (v->pitch < v->W) return fail(LF_EINVAL, "pitch %d < W %d", v->pitch, v->W);
    if (v->channels != 0 && v->channels != 1 && v->channels != 3)
        return fail(LF_EINVAL, "channels=%d (1 or 3)", v->channels);
    return LF_OK;
}

int channels_of(const lf_view_set* v) { return v->channels == 3 ? 3 : 1; }

lf_status check_window(lf_census_window w) {
    if (w.win_h < 1 || w.win_w < 1 || w.win_h % 2 == 0 || w.win_w % 2 == 0)
        return fail(LF_EINVAL, "Census window %dx%d must be odd", w.win_h, w.win_w);
    if (w.n_offsets < 0 || w.n_offsets > LF_MAX_CENSUS_BITS)
        return fail(LF_EINVAL, "Census n_offsets=%d (0..%d)", w.n_offsets, LF_MAX_CENSUS_BITS);
    if (w.n_offsets == 0 && w.win_h * w.win_w - 1 > 64)
        return fail(LF_EINVAL, "Census window %dx%d has more than 64 bits", w.win_h, w.win_w);
    if (w.win_h > 2 * lf::kMaxCensusRadius + 1 || w.win_w > 2 * lf::kMaxCensusRadius + 1)
        return fail(LF_EUNSUPPORTED, "Census window %dx%d (max side %d)", w.win_h, w.win_w,
                    2 * lf::kMaxCensusRadius + 1);
    for (int n = 0; n < w.n_offsets; ++n) {
        const int dy = w.dy[n], dx = w.dx[n];
        if ((dy == 0 && dx == 0) || std::abs(dy) > w.win_h / 2 || std::abs(dx) > w.win_w / 2)
            return fail(LF_EINVAL, "Census offset %d (%d,%d) outside the %dx%d window or at "
                        "the centre", n, dy, dx, w.win_h, w.win_w);
    }
    return LF_OK;
}

lf_status check_sgm(lf_sgm_params p, const char* which) {
    if (p.P1 < 0 || p.P2 < p.P1 || p.P2 > 16383)
        return fail(LF_EINVAL, "%s penalties P1=%d P2=%d (need 0 <= P1 <= P2 <= 16383)", which,
                    p.P1, p.P2);
    if (p.npaths != 8 && p.npaths != 16)
        return fail(LF_EUNSUPPORTED, "%s npaths=%d (8 or 16)", which, p.npaths);
    return LF_OK;
}

float eff_alpha(const lf_params* p, int dtype) {
    return p->alpha > 0.0f ? p->alpha : (dtype == LF_U8 ? 1.0f : 255.0f);
}

lf_status check_params(const lf_params* p) {
    if (!p) return fail(LF_EINVAL, "params is NULL");
    LF_CHECK(check_window(p->census));
    LF_CHECK(check_sgm(p->sgm_init, "initial"));
    LF_CHECK(check_sgm(p->sgm_final, "final"));
    if (p->sgm_init.npaths * (3 * 64 + p->sgm_init.P2) > 65535)
        return fail(LF_EINVAL, "initial P2=%d overflows the 16-bit aggregated Census cost",
                    p->sgm_init.P2);
    if (p->lambda_far < 0) return fail(LF_EINVAL, "lambda_far=%d (need >= 0)", p->lambda_far);
    if (p->phi < 1) return fail(LF_EINVAL, "phi=%d (need >= 1)", p->phi);
    if (p->lambda < -1) return fail(LF_EINVAL, "lambda=%d (need >= 0, or -1: no bounds)", p->lambda);
    if (p->fill_passes < 0 || p->fill_passes > 8)
        return fail(LF_EINVAL, "fill_passes=%d (0..8)", p->fill_passes);
    if (std::isnan(p->edge_tau)) return fail(LF_EINVAL, "edge_tau is NaN");
    if (!(p->alpha <= 0.0f || std::isfinite(p->alpha))) return fail(LF_EINVAL, "alpha");
    if (p->cost_kind != LF_COST_L2 && p->cost_kind != LF_COST_CENSUS)
        return fail(LF_EINVAL, "cost_kind=%d", p->cost_kind);
    if (p->median != 0 && p->median != 3) return fail(LF_EINVAL, "median=%d (0 or 3)", p->median);
    if (p->sum_bits != 16 && p->sum_bits != 32)
        return fail(LF_EINVAL, "sum_bits=%d (16 or 32)", p->sum_bits);
    if (p->sum_bits == 16 && 65535 / p->sgm_final.npaths - p->sgm_final.P2 < 1)
        return fail(LF_EINVAL, "final P2=%d leaves no room in 16-bit sums", p->sgm_final.P2);
    return LF_OK;
}



// Workspace plans -----------------------------------------------------------
struct InitPlan {
    uint64_t* census;     // [1 + nv][C][HW]
    void* paths;          // per-direction path costs of the SGM
    int16_t* maps;        // [nv][HW]
    int16_t* tmp;         // [HW]
};

size_t plan_initial(Carve& c, int S, int T, int C, int H, int W, int N, const lf_params* prm,
                    InitPlan* p) {
    int st[8];
    const int nv = lf::cross_views(S, T, st);
    const size_t HW = (size_t)H * W;
    InitPlan q;
    q.census = (uint64_t*)c.take((1 + nv) * C * HW * sizeof(uint64_t));
    q.paths = c.take(lf::sgm_dense_scratch_bytes(nv, H, W, N, prm->sgm_init.npaths,
                                                 C * lf::census_bits(prm->census),
                                                 prm->sgm_init.P2));
    q.maps = (int16_t*)c.take(nv * HW * sizeof(int16_t));
    q.tmp = (int16_t*)c.take(HW * sizeof(int16_t));
    if (p) *p = q;
    return c.used;
}

struct CostPlan {
    void* scan;           // prefix-sum scratch
    uint64_t* census_all; // [S*T][C][HW] (Census kind only)
    void* padded;         // [S*T][C][H+2][W+2] edge-replicated views (l2 kind only)
};

size_t plan_cost(Carve& c, int S, int T, int C, int H, int W, const lf_params* prm,
                 CostPlan* p) {
    const size_t HW = (size_t)H * W;
    CostPlan q;
    q.scan = c.take(lf::scan_scratch_bytes((int64_t)HW));
    const bool census = prm && prm->cost_kind == LF_COST_CENSUS;
    q.census_all =
        census ? (uint64_t*)c.take((size_t)S * T * C * HW * sizeof(uint64_t)) : nullptr;
    // sized for float32 views (uint8 ones use a quarter of it)
    q.padded =
        census ? nullptr
               : c.take((size_t)S * T * C * (H + lf::kPadH) * (W + lf::kPadW) * sizeof(float));
    if (p) *p = q;
    return c.used;
}

struct DepthPlan {
    int16_t *dinit, *lo, *hi, *d_index;
    int64_t* offsets;
    uint16_t* cost;
    void* csum;
    float* pre_median;
    void* init_ws;
    size_t init_bytes;
    void* cost_ws;
    size_t cost_bytes;
    void* sgm_ws;
    size_t sgm_bytes;
};

size_t plan_depth(void* base, int S, int T, int C, int H, int W, int N, const lf_params* prm,
                  DepthPlan* p) {
    Carve c(base);
    const size_t HW = (size_t)H * W, cells = HW * N;
    DepthPlan q;
    q.dinit = (int16_t*)c.take(HW * 2);
    q.lo = (int16_t*)c.take(HW * 2);
    q.hi = (int16_t*)c.take(HW * 2);
    q.d_index = (int16_t*)c.take(HW * 2);
    q.offsets = (int64_t*)c.take((HW + 1) * 8);
    q.cost = (uint16_t*)c.take(cells * 2);
    q.csum = c.take(cells * (prm->sum_bits == 16 ? 2 : 4));
    q.pre_median = (float*)c.take(lf_wta_workspace_size(H, W));
    // the initial and the cost stage never run at once: they share one region
    Carve ci(nullptr), cc(nullptr);
    q.init_bytes = plan_initial(ci, S, T, C, H, W, N, prm, nullptr);
    q.cost_bytes = plan_cost(cc, S, T, C, H, W, prm, nullptr);
    q.sgm_bytes = lf_sgm_workspace_size(H, W, N, prm->sgm_final.npaths);
    size_t shared = q.init_bytes > q.cost_bytes ? q.init_bytes : q.cost_bytes;
    if (q.sgm_bytes > shared) shared = q.sgm_bytes;
    q.init_ws = c.take(shared);
    q.cost_ws = q.init_ws;
    q.sgm_ws = q.init_ws;
    if (p) *p = q;
    return c.used;
}


lf_status check_initial_size(int H, int W, int N) {
    if ((int64_t)H * W * ((N + 3) / 4 * 4) * 2 >= ((int64_t)1 << 31))
        return fail(LF_EUNSUPPORTED, "H*W*N = %lld cells per view (max 2^30)",
                    (long long)H * W * N);
    return LF_OK;
}

lf_status check_views_size(const lf_view_set* v) {
    const int64_t bytes = (int64_t)v->S * v->T * channels_of(v) * v->H * v->pitch *
                          (v->dtype == LF_U8 ? 1 : 4);
    if (bytes >= ((int64_t)1 << 31))
        return fail(LF_EUNSUPPORTED, "light field of %lld bytes (max 2 GiB)", (long long)bytes);
    return LF_OK;
}

lf_status check_depth_args(const lf_view_set* views, const float* hyp, int N,
                           const lf_params* prm, const float* disparity, const void* ws,
                           size_t ws_bytes) {
    LF_CHECK(check_views(views));
    LF_CHECK(check_shape(views->S, views->T, views->H, views->W, N));
    LF_CHECK(check_params(prm));
    LF_CHECK(check_initial_size(views->H, views->W, N));
    LF_CHECK(check_views_size(views));
    if (!hyp || !disparity || !ws) return fail(LF_EINVAL, "NULL argument");
    const size_t need = plan_depth(nullptr, views->S, views->T, channels_of(views), views->H,
                                   views->W, N, prm, nullptr);
    if (ws_bytes < need) return fail(LF_ENOSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((uintptr_t)ws % kAlign) return fail(LF_EINVAL, "workspace not 256-byte aligned");
    return LF_OK;
}

// The fields of a job that come from the light field and the parameters.
lf::Job base_job(const lf_view_set* v, const float* hyp, int N, const lf_params* prm) {
    lf::Job j{};
    j.views = v->data;
    j.dtype = v->dtype;
    j.S = v->S;
    j.T = v->T;
    j.H = v->H;
    j.W = v->W;
    j.pitch = v->pitch;
    j.C = channels_of(v);
    j.N = N;
    j.hyp = hyp;
    j.prm = *prm;
    j.alpha = eff_alpha(prm, v->dtype);
    j.cap = lf_cost_cap(prm->sgm_final.P2, prm->sgm_final.npaths, prm->sum_bits);
    j.nv = lf::cross_views(v->S, v->T, j.st);
    return j;
}

// A whole-method job over the workspace layout of plan_depth.
lf::Job depth_job(const lf_view_set* v, const float* hyp, int N, const lf_params* prm,
                  float* disparity, int16_t* d_index, void* ws) {
    DepthPlan pl;
    const int C = channels_of(v);
    plan_depth(ws, v->S, v->T, C, v->H, v->W, N, prm, &pl);
    lf::Job j = base_job(v, hyp, N, prm);
    Carve ci(pl.init_ws);
    InitPlan ip;
    plan_initial(ci, v->S, v->T, C, v->H, v->W, N, prm, &ip);
    Carve cc(pl.cost_ws);
    CostPlan cp;
    plan_cost(cc, v->S, v->T, C, v->H, v->W, prm, &cp);
    j.census = ip.census;
    j.paths = ip.paths;
    j.maps = ip.maps;
    j.fill_tmp = ip.tmp;
    j.dinit = pl.dinit;
    j.lo = pl.lo;
    j.hi = pl.hi;
    j.offsets = pl.offsets;
    j.scan = cp.scan;
    j.census_all = cp.census_all;
    j.padded = cp.padded;
    j.cost = pl.cost;
    j.cost_f32 = nullptr;
    j.cap_cells = (int64_t)v->H * v->W * N;
    j.sgm_ws = pl.sgm_ws;
    j.csum = pl.csum;
    j.d_index = d_index ? d_index : pl.d_index;
    j.pre_median = pl.pre_median;
    j.disparity = disparity;
    return j;
}

lf_status run_initial(lf::Runner& r, const lf::Jobs& jobs) {
    {
        prof::Scope _ps(lf::kStCensus, r);
        LF_HIP(lf::stage_census(r, jobs, false), "census");
    }
    for (int part = 0; part < 3; ++part) {
        prof::Scope _ps(lf::kStInitCost + part, r);
        LF_HIP(lf::stage_sgm_initial(r, jobs, part), "initial SGM");
    }
    prof::Scope _ps(lf::kStBorders, r);
    LF_HIP(lf::stage_borders(r, jobs), "fusion/fill/borders");
    return LF_OK;
}

lf_status run_cost(lf::Runner& r, const lf::Jobs& jobs) {
    {
        prof::Scope _ps(lf::kStOffsets, r);
        LF_HIP(lf::stage_offsets(r, jobs), "offsets");
    }
    {
        prof::Scope _ps(lf::kStCostInputs, r);
        LF_HIP(lf::stage_cost_inputs(r, jobs), "cost inputs");
    }
    prof::Scope _ps(lf::kStCost, r);
    LF_HIP(lf::stage_cost(r, jobs), "bounded cost");
    return LF_OK;
}

lf_status run_depth(lf::Runner& r, const lf::Jobs& jobs) {
    // the boundary-less search (lambda < 0) needs no initial map
    lf::Jobs bounded, boundless;
    for (const lf::Job* j : jobs) (j->prm.lambda < 0 ? boundless : bounded).push_back(j);
    if (!bounded.empty()) LF_CHECK(run_initial(r, bounded));
    if (!boundless.empty()) {
        prof::Scope _ps(lf::kStBorders, r);
        LF_HIP(lf::stage_full_range(r, boundless), "full range");
    }
    LF_CHECK(run_cost(r, jobs));
    {
        prof::Scope _ps(lf::kStSgmFinal, r);
        LF_HIP(lf::stage_sgm_final(r, jobs), "bounded SGM");
    }
    prof::Scope _ps(lf::kStWta, r);
    LF_HIP(lf::stage_wta(r, jobs), "wta/subpixel");
    return LF_OK;
}

}  // namespace

extern "C" {

int lf_abi_version(void) { return LF_ABI_VERSION; }

int32_t lf_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> g(prof::mu);
    const int32_t was = prof::on;
    prof::on = on != 0;
    return was;
}

int32_t lf_profile_read(double* ms, int64_t* launches, int32_t n) {
    std::vector<prof::Rec> recs;
    {
        std::lock_guard<std::mutex> g(prof::mu);
        recs.swap(prof::pending);
    }
    for (int i = 0; i < n && i < lf::kNumStages; ++i) {
        if (ms) ms[i] = 0.0;
        if (launches) launches[i] = 0;
    }
    for (const prof::Rec& r : recs) {
        float t = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess &&
            r.stage < n) {
            if (ms) ms[r.stage] += t;
            if (launches) launches[r.stage] += r.launches;
        }
    }
    std::lock_guard<std::mutex> g(prof::mu);
    for (const prof::Rec& r : recs) {
        prof::pool.push_back(r.a);
        prof::pool.push_back(r.b);
    }
    return lf::kNumStages;
}

const char* lf_profile_stage_name(int32_t i) {
    return i >= 0 && i < lf::kNumStages ? prof::kNames[i] : "";
}

const char* lf_last_error(void) { return g_err.c_str(); }

lf_status lf_validate_hypotheses(const float* host_hyp, int32_t N) {
    if (!host_hyp) return fail(LF_EINVAL, "hypotheses pointer is NULL");
    if (N < 2 || N > LF_MAX_HYPOTHESES)
        return fail(N < 2 ? LF_EINVAL : LF_EUNSUPPORTED, "N = %d hypotheses", N);
    for (int k = 0; k < N; ++k) {
        if (!std::isfinite(host_hyp[k])) return fail(LF_EINVAL, "hypothesis %d is not finite", k);
        if (k > 0 && !(host_hyp[k] > host_hyp[k - 1]))
            return fail(LF_EINVAL, "hypotheses must increase strictly (index %d)", k);
    }
    return LF_OK;
}

int32_t lf_cost_cap(int32_t P2_final, int32_t npaths, int32_t sum_bits) {
    int32_t cap = 65535 - 2 * P2_final;
    if (sum_bits == 16 && npaths > 0 && 65535 / npaths - P2_final < cap)
        cap = 65535 / npaths - P2_final;
    return cap;
}

int32_t lf_cross_views(int32_t S, int32_t T, int32_t* st) {
    int tmp[8];
    const int n = lf::cross_views(S, T, tmp);
    if (st)
        for (int i = 0; i < 2 * n; ++i) st[i] = tmp[i];
    return n;
}

lf_status lf_census(const void* img, int32_t dtype, int32_t H, int32_t W, int32_t pitch,
                    lf_census_window win, uint64_t* out, hipStream_t stream) {
    if (!img || !out) return fail(LF_EINVAL, "NULL image or output");
    if (dtype != LF_U8 && dtype != LF_F32) return fail(LF_EINVAL, "dtype %d", dtype);
    if (H < 1 || W < 1 || pitch < W) return fail(LF_EINVAL, "image %dx%d pitch %d", H, W, pitch);
    LF_CHECK(check_window(win));
    lf::Runner r;
    r.stream = stream;
    prof::Scope _ps(lf::kStCensus, r);
    LF_HIP(lf::census_image(r, img, dtype, H, W, pitch, win, out), "lf_census");
    return LF_OK;
}

size_t lf_initial_workspace_size(int32_t S, int32_t T, int32_t C, int32_t H, int32_t W,
                                 int32_t N, const lf_params* prm) {
    if (S < 1 || T < 1 || H < 1 || W < 1 || N < 1) return 0;
    if (!prm || (C != 1 && C != 3)) return 0;
    Carve c(nullptr);
    return plan_initial(c, S, T, C, H, W, N, prm, nullptr);
}

lf_status lf_initial_disparity(const lf_view_set* views, const float* hyp, int32_t N,
                               const lf_params* prm, int16_t* d_maps, int16_t* d_init,
                               int16_t* d_lo, int16_t* d_hi, uint8_t* census_cost,
                               uint16_t* csum_init, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
    LF_CHECK(check_views(views));
    LF_CHECK(check_shape(views->S, views->T, views->H, views->W, N));
    LF_CHECK(check_params(prm));
    LF_CHECK(check_initial_size(views->H, views->W, N));
    if (!hyp || !d_init || !d_lo || !d_hi || !ws) return fail(LF_EINVAL, "NULL argument");
    const int S = views->S, T = views->T, H = views->H, W = views->W;
    Carve sizer(nullptr);
    const int C = channels_of(views);
    const size_t need = plan_initial(sizer, S, T, C, H, W, N, prm, nullptr);
    if (ws_bytes < need) return fail(LF_ENOSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((uintptr_t)ws % kAlign) return fail(LF_EINVAL, "workspace not 256-byte aligned");
    Carve c(ws);
    InitPlan pl;
    plan_initial(c, S, T, C, H, W, N, prm, &pl);

    lf::Job j = base_job(views, hyp, N, prm);
    j.census = pl.census;
    j.paths = pl.paths;
    j.maps = d_maps ? d_maps : pl.maps;
    j.ccv_out = census_cost;
    j.csum_init_out = csum_init;
    j.fill_tmp = pl.tmp;
    j.dinit = d_init;
    j.lo = d_lo;
    j.hi = d_hi;
    lf::Runner r;
    r.stream = stream;
    LF_CHECK(run_initial(r, {&j}));
    return LF_OK;
}

size_t lf_cost_workspace_size(int32_t S, int32_t T, int32_t C, int32_t H, int32_t W,
                              int32_t N, const lf_params* prm) {
    (void)N;
    if (S < 1 || T < 1 || H < 1 || W < 1 || (C != 1 && C != 3)) return 0;
    Carve c(nullptr);
    return plan_cost(c, S, T, C, H, W, prm, nullptr);
}

lf_status lf_cost_volume_bounded(const lf_view_set* views, const float* hyp, int32_t N,
                                 const lf_params* prm, const int16_t* d_lo,
                                 const int16_t* d_hi, int64_t* offsets, uint16_t* cost,
                                 int64_t cap_cells, float* cost_f32, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
    LF_CHECK(check_views(views));
    LF_CHECK(check_shape(views->S, views->T, views->H, views->W, N));
    LF_CHECK(check_params(prm));
    LF_CHECK(check_views_size(views));
    if (!hyp || !d_lo || !d_hi || !offsets || !cost || !ws)
        return fail(LF_EINVAL, "NULL argument");
    const int S = views->S, T = views->T, H = views->H, W = views->W;
    const int64_t HW = (int64_t)H * W;
    if (cap_cells < HW * N)
        return fail(LF_ENOSPACE, "cap_cells %lld < H*W*N = %lld", (long long)cap_cells,
                    (long long)(HW * N));
    Carve sizer(nullptr);
    const int C = channels_of(views);
    const size_t need = plan_cost(sizer, S, T, C, H, W, prm, nullptr);
    if (ws_bytes < need) return fail(LF_ENOSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((uintptr_t)ws % kAlign) return fail(LF_EINVAL, "workspace not 256-byte aligned");
    Carve c(ws);
    CostPlan pl;
    plan_cost(c, S, T, C, H, W, prm, &pl);

    lf::Job j = base_job(views, hyp, N, prm);
    j.lo = const_cast<int16_t*>(d_lo);
    j.hi = const_cast<int16_t*>(d_hi);
    j.offsets = offsets;
    j.scan = pl.scan;
    j.census_all = pl.census_all;
    j.padded = pl.padded;
    j.cost = cost;
    j.cost_f32 = cost_f32;
    j.cap_cells = cap_cells;
    lf::Runner r;
    r.stream = stream;
    LF_CHECK(run_cost(r, {&j}));
    return LF_OK;
}

size_t lf_sgm_workspace_size(int32_t H, int32_t W, int32_t N, int32_t npaths) {
    if (H < 1 || W < 1 || N < 1 || npaths < 1) return 0;
    return align_up(lf::sgm_bounded_scratch_bytes(H, W, N, npaths));
}

lf_status lf_sgm_aggregate(const uint16_t* cost, const int64_t* offsets, const int16_t* d_lo,
                           const int16_t* d_hi, int32_t H, int32_t W, int32_t N,
                           lf_sgm_params sgm, int32_t sum_bits, void* csum, void* ws,
                           size_t ws_bytes, hipStream_t stream) {
    if (!cost || !offsets || !d_lo || !d_hi || !csum || !ws)
        return fail(LF_EINVAL, "NULL argument");
    if (H < 1 || W < 1) return fail(LF_EINVAL, "image %dx%d", H, W);
    if ((int64_t)H * W > (1 << 30) || H > LF_MAX_SIDE || W > LF_MAX_SIDE)
        return fail(LF_EUNSUPPORTED, "image of %d x %d pixels", H, W);
    if (N < 2 || N > LF_MAX_HYPOTHESES)
        return fail(N < 2 ? LF_EINVAL : LF_EUNSUPPORTED, "N = %d", N);
    LF_CHECK(check_sgm(sgm, "aggregate"));
    if (sum_bits != 16 && sum_bits != 32) return fail(LF_EINVAL, "sum_bits=%d", sum_bits);
    if (lf_cost_cap(sgm.P2, sgm.npaths, sum_bits) < 1)
        return fail(LF_EINVAL, "P2=%d leaves no room for costs in %d-bit sums", sgm.P2, sum_bits);
    const size_t need = lf_sgm_workspace_size(H, W, N, sgm.npaths);
    if (ws_bytes < need) return fail(LF_ENOSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if ((uintptr_t)ws % kAlign) return fail(LF_EINVAL, "workspace not 256-byte aligned");
    lf::Job j{};
    j.H = H;
    j.W = W;
    j.N = N;
    j.prm.sgm_final = sgm;
    j.prm.sum_bits = sum_bits;
    j.cost = const_cast<uint16_t*>(cost);
    j.offsets = const_cast<int64_t*>(offsets);
    j.lo = const_cast<int16_t*>(d_lo);
    j.hi = const_cast<int16_t*>(d_hi);
    j.sgm_ws = ws;
    j.csum = csum;
    lf::Runner r;
    r.stream = stream;
    prof::Scope _ps(lf::kStSgmFinal, r);
    LF_HIP(lf::stage_sgm_final(r, {&j}), "bounded SGM");
    return LF_OK;
}

size_t lf_wta_workspace_size(int32_t H, int32_t W) {
    if (H < 1 || W < 1) return 0;
    return align_up((size_t)H * W * sizeof(float));
}

lf_status lf_wta_subpixel(const void* csum, int32_t sum_bits, const int64_t* offsets,
                          const int16_t* d_lo, const int16_t* d_hi, int32_t H, int32_t W,
                          const float* hyp, int32_t N, int32_t median, int16_t* d_index,
                          float* disparity, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!csum || !offsets || !d_lo || !d_hi || !hyp || !d_index || !disparity)
        return fail(LF_EINVAL, "NULL argument");
    if (H < 1 || W < 1) return fail(LF_EINVAL, "image %dx%d", H, W);
    if (N < 2 || N > LF_MAX_HYPOTHESES)
        return fail(N < 2 ? LF_EINVAL : LF_EUNSUPPORTED, "N = %d", N);
    if (sum_bits != 16 && sum_bits != 32) return fail(LF_EINVAL, "sum_bits=%d", sum_bits);
    if (median != 0 && median != 3) return fail(LF_EINVAL, "median=%d", median);
    if (median == 3 && (!ws || ws_bytes < lf_wta_workspace_size(H, W)))
        return fail(LF_ENOSPACE, "workspace %zu < %zu bytes", ws_bytes,
                    lf_wta_workspace_size(H, W));
    lf::Job j{};
    j.H = H;
    j.W = W;
    j.N = N;
    j.hyp = hyp;
    j.prm.sum_bits = sum_bits;
    j.prm.median = median;
    j.csum = const_cast<void*>(csum);
    j.offsets = const_cast<int64_t*>(offsets);
    j.lo = const_cast<int16_t*>(d_lo);
    j.hi = const_cast<int16_t*>(d_hi);
    j.d_index = d_index;
    j.pre_median = (float*)ws;
    j.disparity = disparity;
    lf::Runner r;
    r.stream = stream;
    prof::Scope _ps(lf::kStWta, r);
    LF_HIP(lf::stage_wta(r, {&j}), "wta/subpixel");
    return LF_OK;
}

size_t lf_depth_workspace_size(int32_t S, int32_t T, int32_t C, int32_t H, int32_t W,
                               int32_t N, const lf_params* prm) {
    if (!prm || S < 1 || T < 1 || H < 1 || W < 1 || N < 1 || (C != 1 && C != 3)) return 0;
    return plan_depth(nullptr, S, T, C, H, W, N, prm, nullptr);
}

lf_status lf_depth(const lf_view_set* views, const float* hyp, int32_t N, const lf_params* prm,
                   float* disparity, int16_t* d_index, void* ws, size_t ws_bytes,
                   hipStream_t stream) {
    LF_CHECK(check_depth_args(views, hyp, N, prm, disparity, ws, ws_bytes));
    lf::Job j = depth_job(views, hyp, N, prm, disparity, d_index, ws);
    lf::Runner r;
    r.stream = stream;
    // the boundary-less search has every pixel at the full range, where longer
    // cost slices pay (measured 1.70 vs 1.88 ms per 9x9x512^2 light field)
    if (prm->lambda < 0) r.tune.cost_cpt = 4;
    return run_depth(r, {&j});
}

}  // extern "C"

// --- lf_depth without a caller workspace --------------------------------------------
// The workspace lives in this file-scope device array.  Its name in host code is a
// host-side stand-in, not a device address: the address of each device's copy is
// taken once per device with hipGetSymbolAddress (with that device current) and
// only that address is handed to kernels.  No part of the workspace has to start
// at zero: every byte lf_depth reads is written earlier in the same call, except
// the slack past the last initial path-cost row, which is read and discarded.
namespace {

__device__ __align__(256) uint8_t scratch[LF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// The current device's copy of `scratch`, resolved on its first use.
lf_status scratch_address(void** out) {
    int dev = -1;
    if (hipError_t e = hipGetDevice(&dev); e != hipSuccess) return device_status(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(LF_EUNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)); e != hipSuccess)
            return device_status(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || (uintptr_t)ptr % kAlign) return fail(LF_EDEVICE, "scratch address %p", ptr);
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return LF_OK;
}

}  // namespace

extern "C" lf_status lf_depth_noalloc(const lf_view_set* views, const float* hyp, int32_t N,
                                      const lf_params* prm, float* disparity, int16_t* d_index,
                                      hipStream_t stream) {
    LF_CHECK(check_views(views));
    LF_CHECK(check_shape(views->S, views->T, views->H, views->W, N));
    LF_CHECK(check_params(prm));
    const size_t need = plan_depth(nullptr, views->S, views->T, channels_of(views), views->H,
                                   views->W, N, prm, nullptr);
    if (need > (size_t)LF_NOALLOC_SCRATCH_BYTES)
        return fail(LF_ENOSPACE,
                    "light field needs %zu bytes of workspace; lf_depth_noalloc holds %zu "
                    "(use lf_depth with a caller workspace)",
                    need, (size_t)LF_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    LF_CHECK(scratch_address(&ws));
    return lf_depth(views, hyp, N, prm, disparity, d_index, ws, LF_NOALLOC_SCRATCH_BYTES, stream);
}

// --- used by the batch plan and the request loop ----------------------------------
namespace lf {

lf_status validate_request(const lf_request* q, size_t ws_bytes, const void* ws) {
    if (!q) return fail(LF_EINVAL, "request is NULL");
    if (!ws) {
        LF_CHECK(check_views(&q->views));
        LF_CHECK(check_shape(q->views.S, q->views.T, q->views.H, q->views.W, q->N));
        LF_CHECK(check_params(&q->params));
        LF_CHECK(check_initial_size(q->views.H, q->views.W, q->N));
        LF_CHECK(check_views_size(&q->views));
        if (!q->hyp || !q->disparity) return fail(LF_EINVAL, "NULL argument");
        return LF_OK;
    }
    return check_depth_args(&q->views, q->hyp, q->N, &q->params, q->disparity, ws, ws_bytes);
}

size_t request_workspace_bytes(const lf_request* q) {
    return lf_depth_workspace_size(q->views.S, q->views.T, channels_of(&q->views), q->views.H,
                                   q->views.W, q->N, &q->params);
}

Job request_job(const lf_request* q, void* ws) {
    return depth_job(&q->views, q->hyp, q->N, &q->params, q->disparity, q->d_index, ws);
}

lf_status run_depth_jobs(Runner& r, const Jobs& jobs) { return run_depth(r, jobs); }

lf_status record_error(lf_status s, const char* fmt, const char* what) {
    return fail(s, fmt, what);
}

}  // namespace lf
