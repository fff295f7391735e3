// Per-pixel stages around the two SGM passes (Sec. 3.4-3.6): fusion of the
// intermediate maps, median hole filling, Sobel edge exclusion and the borders
// of Eq. (11), the prefix sum that indexes the bounded volume, WTA with the
// parabola sub-pixel refinement, and the 3x3 median.  All HBM-light: one thread
// per pixel, coalesced along rows.
#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kThreads = 256;

inline dim3 grid1d(int64_t n) { return dim3((unsigned)((n + kThreads - 1) / kThreads)); }

// --- fusion with confidence threshold phi (Sec. 3.4) -----------------------
__global__ __launch_bounds__(kThreads) void fuse_kernel(const int16_t* __restrict__ maps, int nv,
                                                        int HW, int phi,
                                                        int16_t* __restrict__ dinit) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= HW) return;
    int acc = maps[p];
    bool valid = true;
    for (int i = 1; i < nv; ++i) {
        const int di = maps[(size_t)i * HW + p];
        if (valid && abs(acc - di) < phi)
            acc = (acc + di) >> 1;
        else
            valid = false;
    }
    dinit[p] = (int16_t)(valid ? acc : -1);
}

// --- one median hole-filling pass: lower median of the valid 8-neighbours ---
__global__ __launch_bounds__(kThreads) void fill_kernel(const int16_t* __restrict__ in,
                                                        int16_t* __restrict__ out, int H, int W) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= H * W) return;
    const int v = p / W, u = p - v * W;
    const int d0 = in[p];
    if (d0 >= 0) {
        out[p] = (int16_t)d0;
        return;
    }
    // rank-based selection: the lower median of n values is the one with
    // (n-1)/2 values strictly below it and at least (n-1)/2 + 1 at or below it
    int vals[8], n = 0;
    for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j) {
            if (i == 0 && j == 0) continue;
            const int y = v + i, x = u + j;
            if (y < 0 || y >= H || x < 0 || x >= W) continue;
            const int d = in[(size_t)y * W + x];
            if (d >= 0) vals[n++] = d;
        }
    int res = -1;
    const int want = (n - 1) / 2;
    for (int a = 0; a < n; ++a) {
        int below = 0, atmost = 0;
        for (int b = 0; b < n; ++b) {
            below += vals[b] < vals[a];
            atmost += vals[b] <= vals[a];
        }
        if (below <= want && want < atmost) res = vals[a];
    }
    out[p] = (int16_t)res;
}

// --- Sobel edge exclusion and borders, Eq. (11) -----------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void borders_kernel(const int16_t* __restrict__ dinit,
                                                           const T* __restrict__ ref, int pitch,
                                                           int H, int W, int N, int lambda,
                                                           float alpha, float tau,
                                                           int16_t* __restrict__ lo,
                                                           int16_t* __restrict__ hi) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= H * W) return;
    const int v = p / W, u = p - v * W;
    const int ym = max(v - 1, 0), yp = min(v + 1, H - 1);
    const int xm = max(u - 1, 0), xp = min(u + 1, W - 1);
    auto I = [&](int y, int x) { return ld(ref + (size_t)y * pitch + x); };
    const float gx = ((I(ym, xp) + 2.0f * I(v, xp)) + I(yp, xp)) -
                     ((I(ym, xm) + 2.0f * I(v, xm)) + I(yp, xm));
    const float gy = ((I(yp, xm) + 2.0f * I(yp, u)) + I(yp, xp)) -
                     ((I(ym, xm) + 2.0f * I(ym, u)) + I(ym, xp));
    const float g = fabsf(gx) + fabsf(gy);
    const bool edge = alpha * g > tau;
    const int d = dinit[p];
    if (d < 0 || edge) {
        lo[p] = 0;
        hi[p] = (int16_t)(N - 1);
    } else {
        lo[p] = (int16_t)max(d - lambda, 0);
        hi[p] = (int16_t)min(d + lambda, N - 1);
    }
}

// --- exclusive prefix sum of the range widths -> CSR offsets ----------------
constexpr int kScanPerThread = 8;
constexpr int kScanTile = kThreads * kScanPerThread;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t x, int64_t* sh, int64_t& total) {
    // Hillis-Steele over the 256 per-thread partial sums in LDS
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int o = 1; o < kThreads; o <<= 1) {
        const int64_t y = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    total = sh[kThreads - 1];
    const int64_t excl = sh[t] - x;
    __syncthreads();
    return excl;
}

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const int16_t* __restrict__ lo,
                                                               const int16_t* __restrict__ hi,
                                                               int64_t HW,
                                                               int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int i = 0; i < kScanPerThread; ++i) {
        const int64_t p = base + (int64_t)i * kThreads + threadIdx.x;
        if (p < HW) s += (int64_t)(hi[p] - lo[p] + 1);
    }
    int64_t total;
    block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void scan_blocks_kernel(int64_t* __restrict__ bsum,
                                                               int nblocks,
                                                               int64_t* __restrict__ offsets,
                                                               int64_t HW) {
    // single workgroup: exclusive scan of the per-tile totals, in chunks of 256
    __shared__ int64_t sh[kThreads];
    int64_t carry = 0;
    for (int c = 0; c < nblocks; c += kThreads) {
        const int i = c + threadIdx.x;
        const int64_t x = i < nblocks ? bsum[i] : 0;
        int64_t total;
        const int64_t ex = block_exclusive_scan(x, sh, total);
        if (i < nblocks) bsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) offsets[HW] = carry;
}

__global__ __launch_bounds__(kThreads) void scan_apply_kernel(const int16_t* __restrict__ lo,
                                                              const int16_t* __restrict__ hi,
                                                              int64_t HW,
                                                              const int64_t* __restrict__ bsum,
                                                              int64_t* __restrict__ offsets) {
    __shared__ int64_t sh[kThreads];
    // each thread owns kScanPerThread consecutive pixels of the tile
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
    int w[kScanPerThread];
    int64_t s = 0;
    for (int i = 0; i < kScanPerThread; ++i) {
        const int64_t p = base + i;
        w[i] = p < HW ? hi[p] - lo[p] + 1 : 0;
        s += w[i];
    }
    int64_t total;
    int64_t run = bsum[blockIdx.x] + block_exclusive_scan(s, sh, total);
    for (int i = 0; i < kScanPerThread; ++i) {
        const int64_t p = base + i;
        if (p < HW) offsets[p] = run;
        run += w[i];
    }
}

// --- WTA (Eq. 10) and the parabola sub-pixel step (Sec. 3.6) ----------------
template <typename SumT>
__global__ __launch_bounds__(kThreads) void wta_subpixel_kernel(
    const SumT* __restrict__ csum, const int64_t* __restrict__ off,
    const int16_t* __restrict__ lo, const int16_t* __restrict__ hi, int HW,
    const float* __restrict__ hyp, int16_t* __restrict__ d_index, float* __restrict__ disp) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= HW) return;
    const int l = lo[p], h = hi[p];
    const SumT* c = csum + off[p] - l;     // c[k] for k in [l, h]
    int best = l;
    uint32_t bv = c[l];
    for (int k = l + 1; k <= h; ++k) {
        const uint32_t x = c[k];
        if (x < bv) {
            bv = x;
            best = k;
        }
    }
    d_index[p] = (int16_t)best;
    float d = hyp[best];
    if (best - 1 >= l && best + 1 <= h && h - l >= 4) {
        const int64_t cm = c[best - 1], c0 = c[best], cp = c[best + 1];
        const float o = (float)(cm - cp) / (2.0f * (float)(cm + cp - 2 * c0));
        d = o >= 0.0f ? fmaf(o, hyp[best + 1] - hyp[best], hyp[best])
                      : fmaf(o, hyp[best] - hyp[best - 1], hyp[best]);
    }
    disp[p] = d;
}

// --- 3x3 median, clamp-to-edge ----------------------------------------------
__global__ __launch_bounds__(kThreads) void median3_kernel(const float* __restrict__ in,
                                                           float* __restrict__ out, int H, int W) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= H * W) return;
    const int v = p / W, u = p - v * W;
    float w[9];
    int n = 0;
    for (int i = -1; i <= 1; ++i) {
        const int y = clampi(v + i, 0, H - 1);
        for (int j = -1; j <= 1; ++j) w[n++] = in[(size_t)y * W + clampi(u + j, 0, W - 1)];
    }
    // rank selection: the median has at most 4 values below it and at least 5 at or below
    float med = w[4];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        int below = 0, atmost = 0;
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            below += w[b] < w[a];
            atmost += w[b] <= w[a];
        }
        if (below <= 4 && 4 < atmost) med = w[a];
    }
    out[p] = med;
}

}  // namespace

hipError_t launch_fuse(const int16_t* maps, int nv, int HW, int phi, int16_t* dinit,
                       hipStream_t st) {
    hipLaunchKernelGGL(fuse_kernel, grid1d(HW), dim3(kThreads), 0, st, maps, nv, HW, phi, dinit);
    return hipGetLastError();
}

hipError_t launch_fill(const int16_t* in, int16_t* out, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(fill_kernel, grid1d((int64_t)H * W), dim3(kThreads), 0, st, in, out, H, W);
    return hipGetLastError();
}

hipError_t launch_borders(const int16_t* dinit, const void* ref, int dtype, int pitch, int H,
                          int W, int N, int lambda, float alpha, float tau, int16_t* lo,
                          int16_t* hi, hipStream_t st) {
    if (dtype == LF_U8)
        hipLaunchKernelGGL(borders_kernel<uint8_t>, grid1d((int64_t)H * W), dim3(kThreads), 0, st,
                           dinit, (const uint8_t*)ref, pitch, H, W, N, lambda, alpha, tau, lo, hi);
    else
        hipLaunchKernelGGL(borders_kernel<float>, grid1d((int64_t)H * W), dim3(kThreads), 0, st,
                           dinit, (const float*)ref, pitch, H, W, N, lambda, alpha, tau, lo, hi);
    return hipGetLastError();
}

size_t scan_scratch_bytes(int64_t HW) {
    const int64_t nb = (HW + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * sizeof(int64_t);
}

hipError_t launch_offsets(const int16_t* lo, const int16_t* hi, int64_t HW, int64_t* offsets,
                          void* scratch, hipStream_t st) {
    const int nb = (int)((HW + kScanTile - 1) / kScanTile);
    int64_t* bsum = (int64_t*)scratch;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(kThreads), 0, st, lo, hi, HW, bsum);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kThreads), 0, st, bsum, nb, offsets, HW);
    hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(kThreads), 0, st, lo, hi, HW, bsum,
                       offsets);
    return hipGetLastError();
}

hipError_t launch_wta_subpixel(const void* csum, int sum_bits, const int64_t* off,
                               const int16_t* lo, const int16_t* hi, int H, int W,
                               const float* hyp, int16_t* d_index, float* disp,
                               hipStream_t st) {
    const int HW = H * W;
    if (sum_bits == 16)
        hipLaunchKernelGGL(wta_subpixel_kernel<uint16_t>, grid1d(HW), dim3(kThreads), 0, st,
                           (const uint16_t*)csum, off, lo, hi, HW, hyp, d_index, disp);
    else
        hipLaunchKernelGGL(wta_subpixel_kernel<uint32_t>, grid1d(HW), dim3(kThreads), 0, st,
                           (const uint32_t*)csum, off, lo, hi, HW, hyp, d_index, disp);
    return hipGetLastError();
}

hipError_t launch_median3(const float* in, float* out, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(median3_kernel, grid1d((int64_t)H * W), dim3(kThreads), 0, st, in, out, H,
                       W);
    return hipGetLastError();
}

}  // namespace lf
