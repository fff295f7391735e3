// Internal declarations of liblf: the description of one light field's work
// (Job), the way a stage's launches are issued (Runner), and the stage functions
// each kernel file provides to the API layer.  Not part of the ABI.
//
// Every kernel exists in two forms built from one body:
//   Single<A>  one light field, its argument record A passed by value;
//   Group<A>   n light fields, records in device memory, member i owning the
//              virtual blocks [prefix[i], prefix[i+1]) of the launch.
// A launch may have fewer workgroups than virtual blocks; a workgroup then loops
// over them (persistent workgroups).  The single-light-field entry points issue
// Single launches directly; a batch plan records Group launches over all of its
// light fields, one per stage and kernel variant.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <functional>
#include <vector>

#include "../../include/lf.h"

// Pointer fields of the kernels' argument records point into device memory.  On
// the device they convert to pointers in the global address space: a kernel that
// reads its record from a batch plan's table (not from its kernel arguments)
// would otherwise access memory with flat instructions, which count against both
// the vector-memory and the LDS wait counters (every LDS wait would then also wait
// for the stores in flight).  gptr<T> has the layout of a plain pointer.
#if defined(__HIP_DEVICE_COMPILE__)
#define LF_GLOBAL __attribute__((address_space(1)))
#else
#define LF_GLOBAL
#endif

namespace lf {

template <class T>
struct gptr {
    union {
        T* p;                 // as the host writes it
        LF_GLOBAL T* g;       // as the device reads it: no generic-to-global cast
    };                        // that the compiler could fold away
    gptr() = default;
    __host__ __device__ gptr(T* q) : p(q) {}
    __device__ operator LF_GLOBAL T*() const { return g; }
    // explicit casts to another element type keep the address space visible
    template <class U>
    __device__ explicit operator U*() const { return (U*)g; }
};

constexpr uint32_t kInf = 0x3FFFFFFFu;   // +inf of the SGM path recurrences
constexpr int kMaxCensusRadius = 7;      // windows up to 15 x 15
constexpr int kPadH = 2, kPadW = 6;      // rows / columns added to the cost stage's view copy
constexpr int kMaxBatchImages = 16;

// Bits of a Census string with this window (the listed neighbours of a sparse
// window, else every pixel of the dense window but the centre).
inline int census_bits(const lf_census_window& w) {
    return w.n_offsets > 0 ? w.n_offsets : w.win_h * w.win_w - 1;
}

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return min(max(x, lo), hi); }

// Loads one view sample as float (8-bit values convert exactly).
template <typename T> __device__ __forceinline__ float ld(const T* p) { return (float)*p; }

// --- grouped launches --------------------------------------------------------
template <class A> struct Single {
    A a;
    uint32_t total;
};

template <class A> struct Group {
    const A* a;
    const uint32_t* prefix;   // [n + 1]
    int n;
    uint32_t total;
};

// The argument record of virtual block vb, returned by value: a kernel keeps it in
// registers, where global stores cannot invalidate it (read through a pointer
// into the device table, every field would have to be re-read after each store
// that might alias it).  Records are indexed with constant indices only.
template <class A>
__device__ __forceinline__ A member(const Single<A>& s, uint32_t vb, uint32_t& local) {
    local = vb;
    return s.a;
}

// A plan's launch tables are written before its launches and never by a kernel:
// they are read through the constant address space, so that the reads are scalar
// loads the compiler may keep (through a plain global pointer, a store anywhere in
// the kernel would make every later read of the table a vector load).
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* table_ptr(const T* p) {
    return (const __attribute__((address_space(4))) T*)p;
}

template <class A>
__device__ __forceinline__ int group_member(const Group<A>& g, uint32_t vb, uint32_t& local) {
    const auto* prefix = table_ptr(g.prefix);
    int lo = 0, hi = g.n;                     // prefix[lo] <= vb < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= vb) lo = mid; else hi = mid;
    }
    local = vb - prefix[lo];
    return lo;
}

template <class A>
__device__ __forceinline__ A member(const Group<A>& g, uint32_t vb, uint32_t& local) {
    static_assert(sizeof(A) % 4 == 0, "records are copied in 32-bit words");
    const auto* src = table_ptr((const uint32_t*)(g.a + group_member(g, vb, local)));
    A out;
    uint32_t* dst = (uint32_t*)&out;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(A) / 4); ++i) dst[i] = src[i];
    return out;
}

// The record read in place (kernel arguments or the device table), for records
// with tables a kernel indexes at run time, which a register copy cannot hold.
template <class A>
__device__ __forceinline__ const A& member_ref(const Single<A>& s, uint32_t vb, uint32_t& local) {
    local = vb;
    return s.a;
}

template <class A>
__device__ __forceinline__ const A& member_ref(const Group<A>& g, uint32_t vb, uint32_t& local) {
    return g.a[group_member(g, vb, local)];
}

// Tunable schedule parameters.  None of them changes a result.
struct Tuning {
    int cost_cpt = 2;        // cells per thread of the bounded cost kernel (2, 4, 8)
    int cost_stride = 1;     // slices walked per cost workgroup (1, 2, 4)
    int dense_depth = 16;    // steps prefetched by the initial-stage SGM (4, 8, 16)
    int bounded_depth = 4;   // steps prefetched by the bounded SGM, 64 lanes per line (4, 8, 16)
    int bounded_lanes = 64;  // lanes per path line of the bounded SGM (16, 32, 64)
    int bounded_offsets = 32;  // 32: 32-bit offsets where volumes allow; 64: 64-bit always
};

// Stages of the method, in order (also the profiling buckets).
enum Stage { kStCensus, kStInitCost, kStInitPaths, kStInitSum, kStBorders, kStOffsets,
             kStCostInputs, kStCost, kStSgmFinal, kStWta, kNumStages };

// Receives the launches of a batch plan.  table() copies host records into the
// plan's device table and returns their device address.
class Recorder {
public:
    virtual ~Recorder() = default;
    virtual const void* table(const void* host, size_t bytes) = 0;
    virtual void add(int stage, std::function<hipError_t(hipStream_t)> fn) = 0;
};

struct Runner {
    hipStream_t stream = nullptr;   // immediate launches
    Recorder* rec = nullptr;        // non-null: record instead
    Tuning tune;
    int launches = 0;               // kernels launched or recorded so far
};

constexpr size_t kMaxArgRecord = 256;   // bytes of one argument record in a plan table

template <class A>
hipError_t launch(Runner& r, int stage, void (*ks)(Single<A>), void (*kg)(Group<A>),
                  const std::vector<A>& args, const std::vector<uint32_t>& blocks,
                  uint32_t threads, uint32_t grid_cap = 0) {
    static_assert(sizeof(A) <= kMaxArgRecord, "argument record too large for a plan table");
    const int n = (int)args.size();
    if (!r.rec) {
        for (int i = 0; i < n; ++i) {
            if (blocks[i] == 0) continue;
            const uint32_t grid = grid_cap && grid_cap < blocks[i] ? grid_cap : blocks[i];
            Single<A> s{args[i], blocks[i]};
            void* kargs[] = {&s};
            hipError_t e = hipLaunchKernel((const void*)ks, dim3(grid), dim3(threads), kargs, 0,
                                           r.stream);
            if (e != hipSuccess) return e;
            ++r.launches;
        }
        return hipGetLastError();
    }
    std::vector<uint32_t> prefix(n + 1, 0);
    for (int i = 0; i < n; ++i) prefix[i + 1] = prefix[i] + blocks[i];
    const uint32_t total = prefix[n];
    if (total == 0) return hipSuccess;
    Group<A> g;
    g.a = (const A*)r.rec->table(args.data(), n * sizeof(A));
    g.prefix = (const uint32_t*)r.rec->table(prefix.data(), (n + 1) * sizeof(uint32_t));
    g.n = n;
    g.total = total;
    const uint32_t grid = grid_cap && grid_cap < total ? grid_cap : total;
    ++r.launches;
    r.rec->add(stage, [=](hipStream_t st) mutable -> hipError_t {
        void* kargs[] = {&g};
        return hipLaunchKernel((const void*)kg, dim3(grid), dim3(threads), kargs, 0, st);
    });
    return hipSuccess;
}

// --- one light field's work ----------------------------------------------------
// Inputs, parameters and the device buffers every stage reads or writes.  A stage
// uses only the buffers it needs; the others may be null.
struct Job {
    const void* views;        // [T][S][C][H][pitch]
    int dtype, S, T, C, H, W, pitch, N;
    const float* hyp;         // [N]
    lf_params prm;
    float alpha;              // effective cost scale
    int32_t cap;              // saturation of the quantised cost
    int nv;                   // cross views
    int st[8];                // (s, t) of each cross view
    // initial stage
    uint64_t* census;         // [1 + nv][C][H*W]: reference, then the cross views
    void* paths;              // initial SGM scratch (sgm_dense_scratch_bytes)
    int16_t* maps;            // [nv][H*W] D_i
    uint8_t* ccv_out;         // [nv][H*W][N] Census costs of Eq. (7), or null (checking)
    uint16_t* csum_init_out;  // [nv][H*W][N] aggregated initial costs, or null (checking)
    int16_t* fill_tmp;        // [H*W]
    int16_t* dinit;           // [H*W]
    int16_t* lo;              // [H*W]
    int16_t* hi;              // [H*W]
    // bounded stage
    int64_t* offsets;         // [H*W + 1]
    void* scan;               // scan_scratch_bytes(H*W)
    uint64_t* census_all;     // [S*T][C][H*W] (Census cost kind)
    void* padded;             // [S*T][C][H+2][W+2] views with a replicated edge (l2 kind)
    uint16_t* cost;           // [cells]
    float* cost_f32;          // [cells] or null
    int64_t cap_cells;
    void* sgm_ws;             // sgm_bounded_scratch_bytes
    void* csum;               // [cells] uint16 or uint32
    int16_t* d_index;         // [H*W]
    float* pre_median;        // [H*W] (median == 3)
    float* disparity;         // [H*W]
};

using Jobs = std::vector<const Job*>;

int cross_views(int S, int T, int* st);
int dense_np(int N);

// Scratch sizes (bytes).
size_t sgm_dense_scratch_bytes(int nv, int H, int W, int N, int npaths, int bits, int P2);
size_t sgm_bounded_scratch_bytes(int H, int W, int N, int npaths);
size_t scan_scratch_bytes(int64_t HW);

// Census of the reference and cross views (initial) or of all S*T views (into
// census_all, for the Census cost kind).
hipError_t stage_census(Runner& r, const Jobs& jobs, bool all_views);
// A standalone Census transform of one image.
hipError_t census_image(Runner& r, const void* img, int dtype, int H, int W, int pitch,
                        const lf_census_window& win, uint64_t* out);
// Census cost + SGM + WTA over the cross views -> maps.
// part 0: the Census cost volume, 1: the path costs, 2: their sum and the WTA
hipError_t stage_sgm_initial(Runner& r, const Jobs& jobs, int part);
// Fusion, fill passes ending in dinit, edges and borders -> dinit, lo, hi.
hipError_t stage_borders(Runner& r, const Jobs& jobs);
// The full hypothesis range for every pixel -> lo, hi (boundary-less search).
hipError_t stage_full_range(Runner& r, const Jobs& jobs);
// Exclusive prefix sum of the range widths -> offsets.
hipError_t stage_offsets(Runner& r, const Jobs& jobs);
// Bounded matching cost (l2 or Census kind) -> cost (and cost_f32).
hipError_t stage_cost_inputs(Runner& r, const Jobs& jobs);
hipError_t stage_cost(Runner& r, const Jobs& jobs);
// Bounded SGM -> csum.
hipError_t stage_sgm_final(Runner& r, const Jobs& jobs);
// WTA + sub-pixel (+ median) -> d_index, disparity.
hipError_t stage_wta(Runner& r, const Jobs& jobs);

// --- the whole method over jobs (api.hip) --------------------------------------
// Checks a request as lf_depth checks its arguments (ws may be null: then only
// the light field and parameters are checked).
lf_status validate_request(const lf_request* q, size_t ws_bytes, const void* ws);
size_t request_workspace_bytes(const lf_request* q);
Job request_job(const lf_request* q, void* ws);
lf_status run_depth_jobs(Runner& r, const Jobs& jobs);
// Sets the thread's last error (lf_last_error) and returns s.
lf_status record_error(lf_status s, const char* fmt, const char* what);

}  // namespace lf
