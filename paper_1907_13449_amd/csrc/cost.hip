// Bounded matching cost over all views, Sec. 3.5: Eq. (12) (l2 of the
// bilinearly shifted views) and Eq. (15) (Census Hamming at the nearest shift).
//
// Work is flattened over the cells of the CSR volume so that pixels whose range
// is the full hypothesis set and pixels with a 2*lambda+1 window share the
// machine evenly: a 256-thread workgroup owns 64 consecutive pixels, stages their
// offsets and ranges in LDS, and its threads stride over the cells of those
// pixels; a cell finds its pixel by binary search in LDS.  Consecutive threads
// therefore handle consecutive hypotheses of one pixel and then the next pixel
// of the row, so the four bilinear taps of a view are read from a narrow band of
// two rows (L1/L2 resident) and the cost writes are fully coalesced.
//
// The view loop runs t outer, s inner, float32, with the shift of each view and
// hypothesis rounded once: this is the precision the quantised integer cost is
// decided in.  The reference view contributes exactly +0 and is skipped.
#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kPix = 64;        // pixels per workgroup
constexpr int kThreads = 256;

struct CellMap {
    int64_t first;              // first cell of the workgroup
    int64_t end;                // one past its last cell
    int p0;                     // first pixel
};

// Stages offsets/lo of the workgroup's pixels; returns its cell span.
__device__ __forceinline__ CellMap stage_cells(const int64_t* __restrict__ off,
                                               const int16_t* __restrict__ lo, int HW,
                                               int64_t* s_off, int* s_lo) {
    const int p0 = blockIdx.x * kPix;
    const int np = min(kPix, HW - p0);
    for (int i = threadIdx.x; i <= np; i += kThreads) {
        s_off[i] = off[p0 + i];
        if (i < np) s_lo[i] = lo[p0 + i];
    }
    __syncthreads();
    return CellMap{s_off[0], s_off[np], p0};
}

// Largest i with s_off[i] <= c (the pixel that owns cell c).
__device__ __forceinline__ int find_pixel(const int64_t* s_off, int np, int64_t c) {
    int a = 0, b = np;            // invariant: s_off[a] <= c < s_off[b]
    while (b - a > 1) {
        const int mid = (a + b) >> 1;
        if (s_off[mid] <= c) a = mid; else b = mid;
    }
    return a;
}

// ---------------------------------------------------------------------------
// l2 cost, Eq. (12).  Work is dealt in equal slices of cells: workgroup b takes
// the cells [b*kChunk, (b+1)*kChunk) of the CSR volume, whatever pixels they
// belong to, so pixels with the full hypothesis range and pixels with a
// 2*lambda+1 window cost the same per cell and no workgroup is a straggler.
// The first pixel of the slice is found by binary search over the offsets; the
// offsets and lower bounds of the slice's pixels are staged in LDS, and each
// cell finds its pixel there.  Consecutive threads take consecutive cells
// (consecutive hypotheses of a pixel, then the next pixel).
//
// Per view the two taps of a bilinear row, (x0, x0+1), are fetched by one 8-byte
// load (the view pointer is only 4-byte aligned, which global loads allow):
// that halves the gather instructions, whose issue rate -- not bytes -- bounds
// this kernel.  At the image edges a tap is clamped; the pair then starts at
// min(x_a, W-2) and each tap picks its element of the pair.
constexpr int kChunk = 1024;           // cells per workgroup
constexpr int kCPT = kChunk / kThreads;

template <typename T>
struct Pair {
    float lo, hi;
};

template <typename T>
__device__ __forceinline__ Pair<T> ld_pair(const T* p) {
    if constexpr (sizeof(T) == 4) {
        float2 v;
        __builtin_memcpy(&v, p, 8);
        return Pair<T>{v.x, v.y};
    } else {
        uint16_t v;
        __builtin_memcpy(&v, p, 2);
        return Pair<T>{(float)(v & 0xFF), (float)(v >> 8)};
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void cost_l2_kernel(
    const T* __restrict__ views, int S, int T_, int H, int W, int pitch,
    const float* __restrict__ hyp, int N, const int16_t* __restrict__ lo,
    const int64_t* __restrict__ off, float alpha, float cap, uint16_t* __restrict__ cost,
    float* __restrict__ cost_f32, int64_t cap_cells) {
    __shared__ int64_t s_off[kChunk + 1];
    __shared__ int s_lo[kChunk];
    __shared__ int s_p0, s_np;
    const int HW = H * W;
    const int64_t total = min(off[HW], cap_cells);
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    if (c0 >= total) return;                     // uniform: the whole workgroup
    const int64_t c1 = min(c0 + kChunk, total);
    if (threadIdx.x == 0) {
        int a = 0, b = HW;                       // off[a] <= c0 < off[b]
        while (b - a > 1) {
            const int mid = (a + b) >> 1;
            if (off[mid] <= c0) a = mid; else b = mid;
        }
        s_p0 = a;
        s_np = min(kChunk, HW - a);
    }
    __syncthreads();
    const int p0 = s_p0, npx = s_np;
    for (int i = threadIdx.x; i <= npx; i += kThreads) {
        s_off[i] = off[p0 + i];
        if (i < npx) s_lo[i] = lo[p0 + i];
    }
    __syncthreads();
    int np = npx;                                 // pixels that own cells of the slice
    {
        int a = 0, b = npx;                       // largest i with s_off[i] <= c1 - 1
        while (b - a > 1) {
            const int mid = (a + b) >> 1;
            if (s_off[mid] <= c1 - 1) a = mid; else b = mid;
        }
        np = a + 1;
    }
    const int sh = (S - 1) / 2, th = (T_ - 1) / 2;
    const size_t vstride = (size_t)H * pitch;
    const T* __restrict__ refv = views + ((size_t)th * S + sh) * vstride;
    const bool pairs = W >= 2;

    for (int r = 0; r < kCPT; ++r) {
        const int64_t c = c0 + threadIdx.x + (int64_t)r * kThreads;
        if (c >= c1) break;
        const int i = find_pixel(s_off, np, c);
        const int p = p0 + i;
        const int v = p / W, u = p - v * W;
        const int k = s_lo[i] + (int)(c - s_off[i]);
        if ((unsigned)k >= (unsigned)N) continue;      // only for ranges outside [0, N)
        const float d = hyp[k];
        const float ref = ld(refv + (size_t)v * pitch + u);
        float acc = 0.0f;
        for (int t = 0; t < T_; ++t) {
            const float shy = (float)(th - t) * d;
            const float y0 = floorf(shy);
            const float fy = shy - y0;
            const int ya = clampi(v + (int)y0, 0, H - 1), yb = clampi(v + (int)y0 + 1, 0, H - 1);
            const T* __restrict__ vt = views + (size_t)t * S * vstride;
            for (int s = 0; s < S; ++s) {
                if (s == sh && t == th) continue;        // adds exactly +0
                const float shx = (float)(sh - s) * d;
                const float x0 = floorf(shx);
                const float fx = shx - x0;
                const int xa = clampi(u + (int)x0, 0, W - 1), xb = clampi(u + (int)x0 + 1, 0, W - 1);
                const T* __restrict__ vs = vt + (size_t)s * vstride;
                float a, b, cc, e;
                if (pairs) {
                    const int q = min(xa, W - 2);          // xa, xb in {q, q+1}
                    const Pair<T> top = ld_pair(vs + (size_t)ya * pitch + q);
                    const Pair<T> bot = ld_pair(vs + (size_t)yb * pitch + q);
                    a = xa == q ? top.lo : top.hi;
                    b = xb == q ? top.lo : top.hi;
                    cc = xa == q ? bot.lo : bot.hi;
                    e = xb == q ? bot.lo : bot.hi;
                } else {
                    a = ld(vs + (size_t)ya * pitch + xa);
                    b = ld(vs + (size_t)ya * pitch + xb);
                    cc = ld(vs + (size_t)yb * pitch + xa);
                    e = ld(vs + (size_t)yb * pitch + xb);
                }
                const float top = fmaf(fx, b - a, a);
                const float bot = fmaf(fx, e - cc, cc);
                const float val = fmaf(fy, bot - top, top);
                acc = acc + fabsf(ref - val);
            }
        }
        const float q = rintf(alpha * acc);
        cost[c] = (uint16_t)(q > cap ? cap : q);
        if (cost_f32) cost_f32[c] = acc;
    }
}

__global__ __launch_bounds__(kThreads) void cost_census_all_kernel(
    const uint64_t* __restrict__ census, int S, int T_, int H, int W,
    const float* __restrict__ hyp, int N, const int16_t* __restrict__ lo,
    const int64_t* __restrict__ off, uint32_t cap, uint16_t* __restrict__ cost,
    float* __restrict__ cost_f32, int64_t cap_cells) {
    __shared__ int64_t s_off[kPix + 1];
    __shared__ int s_lo[kPix];
    const int HW = H * W;
    const CellMap cm = stage_cells(off, lo, HW, s_off, s_lo);
    const int np = min(kPix, HW - cm.p0);
    const int sh = (S - 1) / 2, th = (T_ - 1) / 2;
    const uint64_t* __restrict__ cref = census + ((size_t)th * S + sh) * HW;
    for (int64_t c = cm.first + threadIdx.x; c < cm.end; c += kThreads) {
        if (c >= cap_cells) break;
        const int i = find_pixel(s_off, np, c);
        const int p = cm.p0 + i;
        const int v = p / W, u = p - v * W;
        const int k = s_lo[i] + (int)(c - s_off[i]);
        if ((unsigned)k >= (unsigned)N) continue;
        const float d = hyp[k];
        const uint64_t r = cref[p];
        uint32_t acc = 0;
        for (int t = 0; t < T_; ++t) {
            const int y = clampi(v + (int)rintf((float)(th - t) * d), 0, H - 1);
            for (int s = 0; s < S; ++s) {
                const int x = clampi(u + (int)rintf((float)(sh - s) * d), 0, W - 1);
                acc += (uint32_t)__popcll(r ^ census[((size_t)t * S + s) * HW + (size_t)y * W + x]);
            }
        }
        cost[c] = (uint16_t)min(acc, cap);
        if (cost_f32) cost_f32[c] = (float)acc;
    }
}

}  // namespace

hipError_t launch_cost_l2(const void* views, int dtype, int S, int T, int H, int W, int pitch,
                          const float* hyp, int N, const int16_t* lo, const int16_t* hi,
                          const int64_t* off, float alpha, int32_t cap, uint16_t* cost,
                          float* cost_f32, int64_t cap_cells, hipStream_t st) {
    (void)hi;
    // worst-case number of slices; those past the device-side cell count exit
    const int64_t slices = ((int64_t)H * W * N + kChunk - 1) / kChunk;
    dim3 grid((unsigned)slices);
    if (dtype == LF_U8)
        hipLaunchKernelGGL(cost_l2_kernel<uint8_t>, grid, dim3(kThreads), 0, st,
                           (const uint8_t*)views, S, T, H, W, pitch, hyp, N, lo, off, alpha,
                           (float)cap, cost, cost_f32, cap_cells);
    else
        hipLaunchKernelGGL(cost_l2_kernel<float>, grid, dim3(kThreads), 0, st,
                           (const float*)views, S, T, H, W, pitch, hyp, N, lo, off, alpha,
                           (float)cap, cost, cost_f32, cap_cells);
    return hipGetLastError();
}

hipError_t launch_cost_census_all(const uint64_t* census_all, int S, int T, int H, int W,
                                  const float* hyp, int N, const int16_t* lo, const int16_t* hi,
                                  const int64_t* off, int32_t cap, uint16_t* cost,
                                  float* cost_f32, int64_t cap_cells, hipStream_t st) {
    (void)hi;
    const int HW = H * W;
    dim3 grid((HW + kPix - 1) / kPix);
    hipLaunchKernelGGL(cost_census_all_kernel, grid, dim3(kThreads), 0, st, census_all, S, T, H,
                       W, hyp, N, lo, off, (uint32_t)cap, cost, cost_f32, cap_cells);
    return hipGetLastError();
}

}  // namespace lf
