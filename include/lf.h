/*
 * lf.h -- C ABI of liblf, the MI355X (gfx950) implementation of the hot path of
 * "Rapid Light Field Depth Estimation with Semi-Global Matching" (Anisimov,
 * Wasenmueller, Stricker, 2019): Census / l2 matching costs over the views of a
 * light field, restricted to per-pixel hypothesis bounds from an initial map,
 * and semi-global matching over them.
 *
 * Conventions shared by every entry point
 *  - Pointers are DEVICE pointers unless the comment says "host".  The caller
 *    allocates every buffer, including the workspace; the library never
 *    allocates or frees device memory inside a compute call.
 *  - Calls are asynchronous on `stream` and never synchronise it; outputs are
 *    valid once the stream's work has completed.  Concurrent calls on one stream
 *    are ordered; calls on different streams must not share output or workspace
 *    buffers.
 *  - Arguments are validated on the host before anything is enqueued.  On a
 *    failed check the call returns LF_EINVAL (or LF_ENOSPACE / LF_EUNSUPPORTED),
 *    enqueues nothing and lf_last_error() describes the reason.  A failed kernel
 *    launch returns LF_EDEVICE.  Nothing aborts the process.
 *  - Light field, Sec. 3.1: views L(u,v,s,t) on an S x T angular grid (s
 *    horizontal, t vertical), stored [T][S][H][pitch], each view row-major.  The
 *    reference view is (s_hat, t_hat) = ((S-1)/2, (T-1)/2); S and T are odd.
 *    Hypothesis d places the match of reference pixel (u,v) in view (s,t) at
 *    (u + (s_hat-s) d, v + (t_hat-t) d), Eq. (1).
 *  - Hypotheses: `hyp` is a device float32 array of N strictly increasing
 *    disparities d_0 < ... < d_{N-1} (checked on the host copy by
 *    lf_validate_hypotheses; a device array is not read back).  2 <= N <= 256.
 *    Disparity indices are int16 in [0, N-1]; -1 marks an invalid pixel.
 *  - Image size: H, W <= LF_MAX_SIDE and H*W <= 2^30 pixels (LF_EUNSUPPORTED
 *    beyond; the kernels address a path step's rows with 32-bit offsets).
 *  - Bounded volumes ("CSR" layout): pixel p = v*W + u owns the index range
 *    [d_lo[p], d_hi[p]] and the cells offsets[p] .. offsets[p+1]-1, cell
 *    offsets[p] + (k - d_lo[p]) holding hypothesis k.  offsets has H*W+1 int64
 *    entries (an exclusive prefix sum of the range widths).
 */
#ifndef LF_H
#define LF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LF_ABI_VERSION 6
#define LF_MAX_HYPOTHESES 256
#define LF_MAX_SIDE 65536

typedef enum {
    LF_OK = 0,
    LF_EINVAL = -1,        /* invalid argument (nothing enqueued) */
    LF_ENOSPACE = -2,      /* a caller buffer or the workspace is too small */
    LF_EDEVICE = -3,       /* a HIP call or kernel launch failed */
    LF_EUNSUPPORTED = -4,  /* valid, but outside what the library implements */
    LF_EBUSY = -5,         /* a queue is full or the object is in use; retry later */
    LF_ETIMEOUT = -6,      /* a wait ended before the work did */
    LF_ECANCELED = -7      /* the work was dropped before it ran */
} lf_status;

typedef enum { LF_U8 = 0, LF_F32 = 1 } lf_dtype;

/* Matching cost of the final (bounded) stage: l2, Eq. (12), or Census, Eq. (15). */
typedef enum { LF_COST_L2 = 0, LF_COST_CENSUS = 1 } lf_cost_kind;

/* A light field resident in device memory. */
typedef struct {
    const void* data;   /* [T][S][C][H][pitch] elements of `dtype`; float32 views
                           must be finite (results for NaN or inf are unspecified) */
    int32_t S, T, H, W;
    int32_t pitch;      /* elements between rows, >= W; planes are H*pitch apart */
    int32_t dtype;      /* lf_dtype */
    int32_t channels;   /* C: 1 (or 0) grayscale, 3 colour (Sec. 3.3: Census per
                           channel with the Hamming distances summed; the l2 cost
                           is the Euclidean norm of the colour difference) */
} lf_view_set;

/* Census window, Sec. 3.2 Eq. (2)-(3): win_h rows x win_w columns, both odd and
 * at most 15.  Bit n of a pixel's string (LSB first) is 1 iff the centre is larger
 * than its n-th neighbour, Eq. (3); neighbours outside the image are clamped to
 * the edge.
 *   n_offsets = 0: the dense window, win_h*win_w - 1 <= 64 neighbours in row-major
 *     order with the centre skipped.
 *   n_offsets = 1..LF_MAX_CENSUS_BITS: a sparse window (Sec. 3.2 notes that one
 *     cuts the comparisons; Sec. 4.3 uses a sparse 7x7 one): neighbour n is at row
 *     offset dy[n], column offset dx[n], with (dy, dx) != (0, 0), |dy| <= win_h/2
 *     and |dx| <= win_w/2 (win_h x win_w bounds the pattern); entries from
 *     n_offsets on are ignored.  Repeated offsets are allowed (equal bits).
 * Invalid windows are rejected with LF_EINVAL (LF_EUNSUPPORTED for a side > 15). */
#define LF_MAX_CENSUS_BITS 64
typedef struct {
    int32_t win_h, win_w;
    int32_t n_offsets;
    int8_t dy[LF_MAX_CENSUS_BITS];
    int8_t dx[LF_MAX_CENSUS_BITS];
} lf_census_window;

/* SGM penalties of Eq. (8) (0 <= P1 <= P2 <= 16383) and the number of path
 * directions: 8 (the axis and diagonal neighbours) or 16 (those and the eight
 * knight moves (+-1,+-2), (+-2,+-1), the paper's setting in Sec. 4.3).  A path of
 * direction r starts at every pixel whose predecessor p - r is outside the
 * image. */
typedef struct { int32_t P1, P2, npaths; } lf_sgm_params;

/* Method parameters (Sec. 4.3 gives the paper's values). */
typedef struct {
    lf_census_window census;   /* window of the initial-stage Census */
    lf_sgm_params sgm_init;    /* SGM of the initial map, Sec. 3.4 */
    lf_sgm_params sgm_final;   /* SGM of the final map, Sec. 3.5 */
    int32_t phi;               /* fusion confidence threshold, in index steps (>= 1) */
    int32_t lambda;            /* border half-width of Eq. (11), in index steps (>= 0);
                                  -1: boundary-less search (Sec. 4.5), every pixel keeps
                                  the full range and lf_depth skips the initial map */
    int32_t fill_passes;       /* median hole-filling passes (0..8) */
    float edge_tau;            /* Sobel |Gx|+|Gy| threshold in 8-bit units; +inf: off */
    float alpha;               /* cost scale to 8-bit units; <= 0 selects 1 (U8) / 255 (F32) */
    int32_t cost_kind;         /* lf_cost_kind of the final stage */
    int32_t median;            /* 0: off, 3: 3x3 median of the final map */
    int32_t sum_bits;          /* 16 or 32: width of the final aggregated cost */
    int32_t lambda_far;        /* depth-adaptive border (Sec. 4.6): if > lambda, the
                                  half-width is lambda_far at index 0 (the smallest
                                  disparity) falling linearly to lambda at N-1,
                                  lambda + ((lambda_far-lambda)(N-1-d) + (N-1)/2)/(N-1);
                                  0 (or <= lambda): lambda everywhere */
} lf_params;

/* ------------------------------------------------------------ utilities */
int lf_abi_version(void);

/* Reason for the last non-LF_OK status returned on this host thread. */
const char* lf_last_error(void);

/* host_hyp: host array of N floats.  LF_OK iff 2 <= N <= LF_MAX_HYPOTHESES and the
 * values are finite and strictly increasing. */
lf_status lf_validate_hypotheses(const float* host_hyp, int32_t N);

/* Cap applied when the final cost is quantised, C = min(rint(alpha*S), cap):
 * cap + 2*P2 <= 65535 keeps 16-bit path costs exact beside the +inf sentinel, and
 * with 16-bit sums npaths*(cap + P2) <= 65535 keeps the sum exact. */
int32_t lf_cost_cap(int32_t P2_final, int32_t npaths, int32_t sum_bits);

/* Number of cross-lying views |V| used by the initial stage (Sec. 3.4) and, in
 * host `st` (may be NULL), their (s,t) pairs: (s_hat,0), (s_hat,T-1), (0,t_hat),
 * (S-1,t_hat) with entries equal to the reference view or repeated dropped. */
int32_t lf_cross_views(int32_t S, int32_t T, int32_t* st);

/* Stage timing for measurement.  lf_profile_enable(1) makes every later call
 * record a HIP event pair on its stream around each group of launches (stages:
 * 0 census, 1 initial Census cost volume, 2 initial path costs, 3 their sum and
 * WTA, 4 fusion/fill/borders, 5 offsets, 6 cost inputs (the edge-replicated view
 * copy, or the Census of every view for the Eq. (15) cost), 7 bounded cost,
 * 8 bounded SGM, 9 WTA/sub-pixel/median); returns the previous setting.
 * lf_profile_read waits for the recorded events, writes per-stage milliseconds
 * and launch counts (host arrays of n entries, either may be NULL), forgets the
 * records and returns the number of stages.  Event objects are created on first
 * use and reused; no device memory is allocated. */
int32_t lf_profile_enable(int32_t on);
int32_t lf_profile_read(double* ms, int64_t* launches, int32_t n);
const char* lf_profile_stage_name(int32_t i);

/* --------------------------------------------------------------- stages */

/* Census transform of one image, Sec. 3.2 Eq. (2)-(3).
 * img: [H][pitch] elements of dtype.  out: [H][W] uint64 bit strings. */
lf_status lf_census(const void* img, int32_t dtype, int32_t H, int32_t W, int32_t pitch,
                    lf_census_window win, uint64_t* out, hipStream_t stream);

/* Bytes of workspace lf_initial_disparity needs (C: channels, 1 or 3). */
size_t lf_initial_workspace_size(int32_t S, int32_t T, int32_t C, int32_t H, int32_t W,
                                 int32_t N, const lf_params* prm);

/* Initial disparity map and borders, Sec. 3.4:
 *  1. Census of the reference and cross views;
 *  2. per cross view i, the Census cost of Eq. (7) over all N hypotheses (match
 *     position of Eq. (1) rounded to the nearest pixel, half to even, clamped),
 *     SGM over npaths directions, Eq. (8)-(9), WTA, Eq. (10), lowest index on
 *     ties -> D_i;
 *  3. fusion with threshold phi (running floored average, invalid is final),
 *     `fill_passes` median hole-filling passes (lower median of the valid
 *     8-neighbours), Sobel edge exclusion, borders of Eq. (11) saturated to
 *     [0, N-1]; invalid and edge pixels get the full range.
 * d_maps: [|V|][H][W] int16 or NULL; d_init, d_lo, d_hi: [H][W] int16.
 * census_cost, csum_init: optional outputs for checking (NULL skips them; asking
 * for them adds copy kernels, it changes no other output):
 *   census_cost [|V|][H][W][N] uint8: C_i(p,k) of Eq. (7) (channels summed);
 *   csum_init   [|V|][H][W][N] uint16: the aggregated cost of Eq. (9) from which
 *               D_i is taken, path costs in the normalised form of Eq. (8)
 *               (m = min_j L_r(p-r,j) subtracted at every step; the first pixel of
 *               a path takes L_r = C).
 * ws: at least lf_initial_workspace_size() bytes, 256-byte aligned. */
lf_status lf_initial_disparity(const lf_view_set* views, const float* hyp, int32_t N,
                               const lf_params* prm, int16_t* d_maps, int16_t* d_init,
                               int16_t* d_lo, int16_t* d_hi, uint8_t* census_cost,
                               uint16_t* csum_init, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/* Bytes of workspace lf_cost_volume_bounded needs (prefix-sum scratch, and the
 * Census strings of every view for LF_COST_CENSUS). */
size_t lf_cost_workspace_size(int32_t S, int32_t T, int32_t C, int32_t H, int32_t W,
                              int32_t N, const lf_params* prm);

/* Bounded matching cost over all views, Sec. 3.5:
 *  offsets <- exclusive prefix sum of the widths d_hi - d_lo + 1 ([H*W+1] int64);
 *  for every cell (p, k), k in [d_lo[p], d_hi[p]]:
 *   LF_COST_L2, Eq. (12): S = sum_t sum_s |L_ref(p) - B_{s,t}(p + shift)| in
 *     float32, t outer, s inner, from +0; shift sh = (float)(s_hat-s)*d_k and
 *     likewise for t, bilinear B with x0 = floor(sh), fx = sh - x0,
 *     top = fma(fx,b-a,a), bot = fma(fx,e-c,c), val = fma(fy,bot-top,top), taps
 *     clamped to the image (the reference view adds exactly 0 and is skipped);
 *     cost = min(rint(alpha*S), cap) with alpha*S and rint in float32.
 *   LF_COST_CENSUS, Eq. (15): S = sum over views of the Hamming distance at the
 *     nearest shift; cost = min(S, cap).
 *  cap = lf_cost_cap(prm->sgm_final.P2, prm->sgm_final.npaths, prm->sum_bits).
 * cost: uint16 [cap_cells]; cost_f32: float [cap_cells] or NULL (raw S before
 * quantisation, for checking).  cap_cells must be >= H*W*N (the count is only
 * known on the device), else LF_ENOSPACE. */
lf_status lf_cost_volume_bounded(const lf_view_set* views, const float* hyp, int32_t N,
                                 const lf_params* prm, const int16_t* d_lo,
                                 const int16_t* d_hi, int64_t* offsets, uint16_t* cost,
                                 int64_t cap_cells, float* cost_f32, void* ws,
                                 size_t ws_bytes, hipStream_t stream);

/* Bytes of workspace lf_sgm_aggregate needs: npaths * H*W*N 16-bit path costs
 * (every direction keeps its own path costs; they are summed at the end). */
size_t lf_sgm_workspace_size(int32_t H, int32_t W, int32_t N, int32_t npaths);

/* SGM over a bounded volume, Eq. (8)-(9), on the per-pixel ranges (Sec. 3.5):
 * path costs are computed in the normalised form L_r(p,k) = C(p,k) +
 * min(L_r(p-r,k), L_r(p-r,k+-1) + P1, m + P2) - m with m = min_j L_r(p-r,j) over
 * the range of p-r; terms whose index lies outside that range are omitted; the
 * first pixel of a path takes L_r = C.  csum[cell] = sum over directions.
 * cost: uint16 [cells], every value <= lf_cost_cap(sgm.P2, sgm.npaths, sum_bits)
 * (the caller's contract; lf_cost_volume_bounded guarantees it).
 * Bounds contract (device data, not checked on the host): 0 <= d_lo[p] <= d_hi[p]
 * < N for every pixel and offsets = the exclusive prefix sum of d_hi - d_lo + 1,
 * as lf_initial_disparity and lf_cost_volume_bounded produce them; the cell count
 * offsets[H*W] is then <= H*W*N.  The kernels clamp the count to H*W*N; other
 * breaches give unspecified results.
 * csum: uint16 (sum_bits 16) or uint32 (32) [cells], CSR layout of `cost`.
 * ws: at least lf_sgm_workspace_size() bytes. */
lf_status lf_sgm_aggregate(const uint16_t* cost, const int64_t* offsets, const int16_t* d_lo,
                           const int16_t* d_hi, int32_t H, int32_t W, int32_t N,
                           lf_sgm_params sgm, int32_t sum_bits, void* csum, void* ws,
                           size_t ws_bytes, hipStream_t stream);

/* Bytes of workspace lf_wta_subpixel needs. */
size_t lf_wta_workspace_size(int32_t H, int32_t W);

/* WTA, sub-pixel refinement and median, Sec. 3.5-3.6:
 *  d_index[p] = lowest k in [d_lo, d_hi] minimising csum (Eq. 10);
 *  with c-, c0, c+ the sums at k*-1, k*, k*+1, if k*-1 >= d_lo, k*+1 <= d_hi and
 *  d_hi - d_lo >= 4: o = (float)(c- - c+) / (2*(float)(c- + c+ - 2 c0)) (the
 *  parabola vertex; Eq. (13) as printed has the sign of the denominator
 *  reversed), disparity = o >= 0 ? fma(o, d[k*+1]-d[k*], d[k*])
 *                                : fma(o, d[k*]-d[k*-1], d[k*]); else d[k*];
 *  median = 3: the 3x3 median (clamp-to-edge) of that map.
 * d_index: [H][W] int16; disparity: [H][W] float32.
 * Bounds contract as for lf_sgm_aggregate; bounds outside [0, N-1] are clamped
 * into it (no hypothesis outside the array is read; results are unspecified). */
lf_status lf_wta_subpixel(const void* csum, int32_t sum_bits, const int64_t* offsets,
                          const int16_t* d_lo, const int16_t* d_hi, int32_t H, int32_t W,
                          const float* hyp, int32_t N, int32_t median, int16_t* d_index,
                          float* disparity, void* ws, size_t ws_bytes, hipStream_t stream);

/* Bytes of workspace lf_depth needs (every stage's buffers, including a
 * worst-case H*W*N bounded volume). */
size_t lf_depth_workspace_size(int32_t S, int32_t T, int32_t C, int32_t H, int32_t W,
                               int32_t N, const lf_params* prm);

/* The whole method on one light field: lf_initial_disparity ->
 * lf_cost_volume_bounded -> lf_sgm_aggregate -> lf_wta_subpixel.
 * disparity: [H][W] float32; d_index: [H][W] int16 (the WTA index of the final
 * stage, before sub-pixel refinement) or NULL. */
lf_status lf_depth(const lf_view_set* views, const float* hyp, int32_t N,
                   const lf_params* prm, float* disparity, int16_t* d_index, void* ws,
                   size_t ws_bytes, hipStream_t stream);


/* lf_depth for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same method
 * and the same results as lf_depth, with the workspace taken from a static device
 * array of LF_NOALLOC_SCRATCH_BYTES (64 MiB) that the library holds on every GPU it
 * runs on until the process ends.  The caller still passes the inputs and outputs.
 * A light field whose lf_depth_workspace_size exceeds that returns LF_ENOSPACE
 * (nothing enqueued).  The array's address is resolved on the first call on each
 * device, with that device current; `stream` must belong to the current device.
 * All calls on one GPU share its array: calls that overlap in time on one GPU
 * (different streams, or different host threads) race and give undefined results;
 * calls ordered on one stream are safe.  No device memory is allocated or freed. */
#define LF_NOALLOC_SCRATCH_BYTES (64u << 20)
lf_status lf_depth_noalloc(const lf_view_set* views, const float* hyp, int32_t N,
                           const lf_params* prm, float* disparity, int16_t* d_index,
                           hipStream_t stream);

/* ------------------------------------------------------------- batches
 * Many light fields of uneven resolution, view count and hypothesis range run
 * together: every stage of the method is ONE grouped launch over all of them
 * (one launch per kernel variant: view type, hypotheses per lane, cost kind,
 * sum width), and the whole sequence can be captured once into a HIP graph and
 * replayed with a single graph launch.  Results are identical to lf_depth on
 * each light field alone, for every tuning. */

/* One light field and its outputs. */
typedef struct {
    lf_view_set views;
    const float* hyp;       /* [N] device */
    int32_t N;
    lf_params params;
    float* disparity;       /* [H][W] float32 output */
    int16_t* d_index;       /* [H][W] int16 output, or NULL */
} lf_request;

/* Schedule parameters of the kernels; none changes a result.  0 selects the
 * default.  cost_cells_per_thread: 2 (default; lf_depth takes 4 for the
 * boundary-less search, lambda < 0), 4 or 8 -- cells per thread of
 * one slice of the bounded cost kernel; cost_stride: 1 (default), 2 or 4 --
 * slices each cost workgroup walks (persistent workgroups); dense_prefetch: 4, 8
 * or 16 (default) -- path steps of cost loads in flight per wave in the initial
 * SGM, also the steps whose path costs it stages before copying them out;
 * bounded_prefetch: 4 (default), 8 or 16 -- pixel metadata steps in flight
 * per wave in the bounded SGM with 64 lanes per line (their costs run half as
 * many steps ahead); bounded_lanes: 16, 32 or 64 (default) -- lanes per path line
 * of the bounded SGM (the wavefront-to-path schedule: 64/bounded_lanes lines per
 * wave, a line's range covered in chunks of that many hypotheses);
 * bounded_offsets: 32 (default) or 64 -- the bounded SGM with 64 lanes per line
 * addresses its volumes with 32-bit offsets where their worst-case size is below
 * 2^31 bytes and with 64-bit addresses otherwise; 64 takes the 64-bit form
 * everywhere (the form of very large volumes, selectable for testing). */
typedef struct {
    int32_t cost_cells_per_thread;
    int32_t cost_stride;
    int32_t dense_prefetch;
    int32_t bounded_prefetch;
    int32_t bounded_lanes;
    int32_t bounded_offsets;
} lf_tuning;

typedef struct lf_plan lf_plan;

/* Workspace bytes of a batch: each light field's lf_depth workspace plus the
 * plan's device tables.  reqs: host array of n >= 1 requests (only shapes and
 * parameters are read).  Returns 0 for an invalid batch. */
size_t lf_batch_workspace_size(const lf_request* reqs, int32_t n);

/* Plans a batch over the caller's workspace (>= lf_batch_workspace_size bytes,
 * 256-byte aligned) and enqueues the upload of its launch tables on `stream`.
 * reqs is copied; its buffers must stay valid while the plan is used.  tuning
 * may be NULL (defaults).  Validates every request as lf_depth does; on failure
 * nothing is enqueued and *plan is NULL. */
lf_status lf_plan_create(const lf_request* reqs, int32_t n, void* ws, size_t ws_bytes,
                         const lf_tuning* tuning, hipStream_t stream, lf_plan** plan);

/* Times each candidate schedule on the plan's own light fields (running the
 * batch several times, `reps` timed runs per candidate, blocking) and keeps the
 * fastest per stage; writes the choice to `chosen` (host, may be NULL).  Drops a
 * captured graph.  The outputs hold the batch's results afterwards. */
lf_status lf_plan_autotune(lf_plan* plan, hipStream_t stream, int32_t reps, lf_tuning* chosen);

/* Captures the plan's launches into a HIP graph (once; later runs replay it). */
lf_status lf_plan_capture(lf_plan* plan);

/* Runs the batch on `stream`: one graph launch if captured, else the grouped
 * launches one by one.  Must be ordered after the table upload of
 * lf_plan_create / lf_plan_autotune (same stream, or synchronised). */
lf_status lf_plan_run(lf_plan* plan, hipStream_t stream);

/* Kernel launches per run (host), and the tuning in use. */
int32_t lf_plan_launches(const lf_plan* plan);
lf_status lf_plan_tuning(const lf_plan* plan, lf_tuning* out);

/* Frees the plan's host memory and graph.  The caller keeps the workspace; work
 * already enqueued must have completed before the workspace is reused. */
void lf_plan_destroy(lf_plan* plan);

/* -------------------------------------------------------- request loop
 * A server that admits light fields as they arrive and runs them on the device
 * with continuous batching: a scheduler thread admits pending requests whose
 * workspace fits in the free part of a caller-provided device arena (first fit,
 * later requests may pass one that does not fit yet), groups those admitted
 * together into one batch plan and launches it on one of its streams while
 * earlier batches are still running; when a batch completes its memory returns
 * to the arena and waiting requests are admitted.  A batch of one runs the
 * lf_depth launches directly (no plan, no table upload).  At most max_large
 * large requests run at once; smaller ones run beside them.  The arena (cost and
 * aggregation buffers included) stays resident for the server's life. */

typedef struct lf_server lf_server;

typedef struct {
    void* arena;                /* device memory owned by the caller, 256-byte aligned */
    size_t arena_bytes;
    int32_t max_batch;          /* light fields per batch (>= 1) */
    int32_t max_inflight;       /* batches on the device at once (1..4); one stream each */
    int32_t max_queue;          /* pending requests before lf_server_submit says LF_EBUSY */
    int32_t group_ratio;        /* 0: any mix; r >= 2: a batch only takes requests whose
                                   workspace is within a factor r of its first member's
                                   (similar sizes: a small request does not wait for a
                                   large one's batch) */
    lf_tuning tuning;           /* schedule of every batch (zeros: defaults) */
    int64_t large_bytes;        /* a request whose workspace exceeds this is "large" (it
                                   fills the GPU by itself); 0: 256 MiB */
    int32_t max_large;          /* large requests on the device at once (two would only
                                   share the GPU and both finish late); 0: 1 */
} lf_server_config;

/* Times of one request on the host steady clock, in seconds since the server
 * was created, and the batch it ran in. */
typedef struct {
    double t_submit, t_admit, t_launch, t_done;
    int64_t batch;              /* sequence number of its batch */
    int32_t batch_size;         /* light fields in that batch */
    int32_t status;             /* lf_status of the request */
} lf_request_info;

/* Creates the server and its scheduler thread (streams are created on first
 * use, at default priority). */
lf_status lf_server_create(const lf_server_config* cfg, lf_server** out);

/* Queues a request (copied; its buffers must stay valid until it completes).
 * Ordering: the request's device work starts only after everything enqueued on
 * `stream` before this call (the producer of its views and hypotheses, earlier
 * users of its outputs) has completed: an event is recorded on `stream` here and
 * the batch's stream waits for it.  NULL is the null stream.
 * If the event cannot be recorded the request completes with LF_EDEVICE.
 * Returns LF_EINVAL for an invalid request, LF_ENOSPACE if its workspace can
 * never fit in the arena, LF_EBUSY if the queue is full; *ticket identifies it. */
lf_status lf_server_submit(lf_server* srv, const lf_request* req, hipStream_t stream,
                           int64_t* ticket);

/* Waits up to timeout_s seconds (< 0: forever) for a ticket; on completion
 * returns the request's status (LF_OK when its outputs are ready) and fills
 * *info (host, may be NULL), and forgets the ticket.  LF_ETIMEOUT if it is still
 * running, LF_EINVAL for an unknown ticket. */
lf_status lf_server_wait(lf_server* srv, int64_t ticket, double timeout_s, lf_request_info* info);

/* Counters (host, any may be NULL): requests completed, batches launched, bytes
 * of the arena in use now, and the most ever in use. */
void lf_server_stats(const lf_server* srv, int64_t* completed, int64_t* batches,
                     int64_t* arena_in_use, int64_t* arena_peak);

/* Stops the scheduler: requests not yet launched complete with LF_ECANCELED,
 * batches on the device are waited for; then frees the server. */
void lf_server_destroy(lf_server* srv);

#ifdef __cplusplus
}
#endif
#endif
