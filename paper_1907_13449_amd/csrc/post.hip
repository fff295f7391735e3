// Per-pixel stages around the two SGM passes (Sec. 3.4-3.6): fusion of the
// intermediate maps, median hole filling, Sobel edge exclusion and the borders
// of Eq. (11), the prefix sum that indexes the bounded volume, WTA with the
// parabola sub-pixel refinement, and the 3x3 median.  All HBM-light: one thread
// per pixel, coalesced along rows.
#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kThreads = 256;

uint32_t blocks_for(int64_t n) { return (uint32_t)((n + kThreads - 1) / kThreads); }

// --- fusion with confidence threshold phi (Sec. 3.4) -----------------------
struct FuseArgs {
    gptr<const int16_t> maps;      // [nv][HW]
    gptr<int16_t> dinit;
    int nv, HW, phi;
};

template <class Src>
__global__ __launch_bounds__(kThreads) void fuse_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const FuseArgs& a = member(src, vb, b);
        const int p = (int)b * kThreads + threadIdx.x;
        if (p >= a.HW) continue;
        int d[4];                                 // |V| <= 4: all loads in flight at once
#pragma unroll
        for (int i = 0; i < 4; ++i) d[i] = i < a.nv ? a.maps[(size_t)i * a.HW + p] : 0;
        int acc = d[0];
        bool valid = true;
#pragma unroll
        for (int i = 1; i < 4; ++i) {
            if (i >= a.nv) break;
            if (valid && abs(acc - d[i]) < a.phi)
                acc = (acc + d[i]) >> 1;
            else
                valid = false;
        }
        a.dinit[p] = (int16_t)(valid ? acc : -1);
    }
}

// --- one median hole-filling pass: lower median of the valid 8-neighbours ---
struct FillArgs {
    gptr<const int16_t> in;
    gptr<int16_t> out;
    int H, W;
};

__device__ __forceinline__ void fill_pixel(const FillArgs& a, int p) {
    const int H = a.H, W = a.W;
    const int v = p / W, u = p - v * W;
    const int d0 = a.in[p];
    if (d0 >= 0) {
        a.out[p] = (int16_t)d0;
        return;
    }
    // the 8 neighbours in fixed slots, invalid or outside ones as a sentinel above
    // every index; a sorting network (Batcher's odd-even merge, 19 comparators)
    // moves the n valid values to the front in order, and the lower median is
    // the one at (n-1)/2
    constexpr int kNone = 0x7FFF;
    int s[8], n = 0;
#pragma unroll
    for (int i = 0, q = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (i == 1 && j == 1) continue;
            const int y = v + i - 1, x = u + j - 1;
            const int d = y < 0 || y >= H || x < 0 || x >= W ? -1 : a.in[(size_t)y * W + x];
            s[q++] = d >= 0 ? d : kNone;
            n += d >= 0;
        }
    constexpr int kNet[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6},
                                 {5, 7}, {1, 2}, {5, 6}, {0, 4}, {1, 5}, {2, 6}, {3, 7},
                                 {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
    for (int c = 0; c < 19; ++c) {
        const int x = s[kNet[c][0]], y = s[kNet[c][1]];
        s[kNet[c][0]] = min(x, y);
        s[kNet[c][1]] = max(x, y);
    }
    const int want = (n - 1) / 2;
    int res = -1;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (n > 0 && i == want) res = s[i];
    a.out[p] = (int16_t)res;
}

template <class Src>
__global__ __launch_bounds__(kThreads) void fill_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const FillArgs& a = member(src, vb, b);
        const int p = (int)b * kThreads + threadIdx.x;
        if (p < a.H * a.W) fill_pixel(a, p);
    }
}

// --- Sobel edge exclusion and borders, Eq. (11) -----------------------------
struct BordersArgs {
    gptr<const int16_t> dinit;
    gptr<const void> ref;          // C planes of H x pitch
    gptr<int16_t> lo;
    gptr<int16_t> hi;
    int pitch, H, W, N, lambda, lambda_far, C;
    float alpha, tau;
};

// Half-width at initial index d (Sec. 4.6): lambda_far at index 0 (the smallest
// disparity, the farthest point) falling linearly to lambda at N-1, rounded
// half up; lambda_far <= lambda keeps lambda.
__device__ __forceinline__ int border_width(int lambda, int lambda_far, int d, int N) {
    if (lambda_far <= lambda || N < 2) return lambda;
    return lambda + ((lambda_far - lambda) * (N - 1 - d) + (N - 1) / 2) / (N - 1);
}

// d: the filled initial index of pixel p (dinit[p])
template <typename T>
__device__ __forceinline__ void borders_pixel(const BordersArgs& a, int p, int d) {
    const int H = a.H, W = a.W;
    const T* __restrict__ ref = (const T*)a.ref;
    const int v = p / W, u = p - v * W;
    const int ym = max(v - 1, 0), yp = min(v + 1, H - 1);
    const int xm = max(u - 1, 0), xp = min(u + 1, W - 1);
    float g = 0.0f;                               // colour: the strongest channel
    for (int c = 0; c < a.C; ++c) {
        const T* __restrict__ img = ref + (size_t)c * H * a.pitch;
        auto I = [&](int y, int x) { return ld(img + (size_t)y * a.pitch + x); };
        const float gx = ((I(ym, xp) + 2.0f * I(v, xp)) + I(yp, xp)) -
                         ((I(ym, xm) + 2.0f * I(v, xm)) + I(yp, xm));
        const float gy = ((I(yp, xm) + 2.0f * I(yp, u)) + I(yp, xp)) -
                         ((I(ym, xm) + 2.0f * I(ym, u)) + I(ym, xp));
        const float gc = fabsf(gx) + fabsf(gy);
        g = gc > g ? gc : g;
    }
    const bool edge = a.alpha * g > a.tau;
    if (a.lambda < 0 || d < 0 || edge) {          // lambda < 0: boundary-less search
        a.lo[p] = 0;
        a.hi[p] = (int16_t)(a.N - 1);
    } else {
        const int lam = border_width(a.lambda, a.lambda_far, d, a.N);
        a.lo[p] = (int16_t)max(d - lam, 0);
        a.hi[p] = (int16_t)min(d + lam, a.N - 1);
    }
}

template <class Src, typename T>
__global__ __launch_bounds__(kThreads) void borders_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const BordersArgs& a = member(src, vb, b);
        const int p = (int)b * kThreads + threadIdx.x;
        if (p < a.H * a.W) borders_pixel<T>(a, p, a.dinit[p]);
    }
}

// --- fusion, hole filling and borders in one launch -------------------------
// A workgroup owns a 32 x 8 tile of pixels.  It fuses the cross views' maps over
// the tile plus a halo of F = fill_passes pixels into LDS, runs the F Jacobi
// fill passes there (pass f is exact on the tile grown by F - f, since a pass
// reads only the 8 neighbours), and then applies the Sobel test and Eq. (11) to
// its own pixels: the same values as the fuse / fill / borders kernels, with no
// round trips of the intermediate maps and one launch instead of 2 + F.
// Halo positions outside the image read as invalid (-1), which the fill treats
// as it treats a missing neighbour.
constexpr int kPrepTX = 32, kPrepTY = 8, kMaxPrepFill = 3;
constexpr int kPrepMax = (kPrepTX + 2 * kMaxPrepFill) * (kPrepTY + 2 * kMaxPrepFill);

struct PrepArgs {
    FuseArgs fuse;            // fuse.dinit: the filled map (dinit)
    BordersArgs brd;
    int fill;                 // passes, <= kMaxPrepFill
    int tx;                   // tiles along x
};

template <class Src, typename T>
__global__ __launch_bounds__(kThreads) void prep_kernel(Src src) {
    __shared__ int16_t buf[2][kPrepMax];
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const PrepArgs& a = member(src, vb, b);
        const int H = a.brd.H, W = a.brd.W, F = a.fill;
        const int by = (int)b / a.tx, bx = (int)b - by * a.tx;
        const int EW = kPrepTX + 2 * F, EH = kPrepTY + 2 * F;
        const int x0 = bx * kPrepTX - F, y0 = by * kPrepTY - F;
        __syncthreads();                          // LDS of the previous tile is read
        for (int i = threadIdx.x; i < EW * EH; i += kThreads) {
            const int ey = i / EW, ex = i - ey * EW;
            const int y = y0 + ey, x = x0 + ex;
            int out = -1;
            if (y >= 0 && y < H && x >= 0 && x < W) {
                const int p = y * W + x;
                const FuseArgs& f = a.fuse;
                int d[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) d[v] = v < f.nv ? f.maps[(size_t)v * f.HW + p] : 0;
                int acc = d[0];
                bool valid = true;
#pragma unroll
                for (int v = 1; v < 4; ++v) {
                    if (v >= f.nv) break;
                    if (valid && abs(acc - d[v]) < f.phi)
                        acc = (acc + d[v]) >> 1;
                    else
                        valid = false;
                }
                out = valid ? acc : -1;
            }
            buf[0][i] = (int16_t)out;
        }
        __syncthreads();
        int cur = 0;
        for (int pass = 1; pass <= F; ++pass) {
            const int16_t* in = buf[cur];
            int16_t* o = buf[cur ^ 1];
            for (int i = threadIdx.x; i < EW * EH; i += kThreads) {
                const int ey = i / EW, ex = i - ey * EW;
                if (ey < pass || ey >= EH - pass || ex < pass || ex >= EW - pass) continue;
                const int d0 = in[i];
                const int y = y0 + ey, x = x0 + ex;
                if (d0 >= 0 || y < 0 || y >= H || x < 0 || x >= W) {
                    o[i] = (int16_t)d0;               // outside the image: stays absent (-1)
                    continue;
                }
                // lower median of the valid neighbours (as fill_pixel)
                constexpr int kNone = 0x7FFF;
                int sv[8], n = 0;
#pragma unroll
                for (int dy = 0, q = 0; dy < 3; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        if (dy == 1 && dx == 1) continue;
                        const int d = in[i + (dy - 1) * EW + dx - 1];
                        sv[q++] = d >= 0 ? d : kNone;
                        n += d >= 0;
                    }
                constexpr int kNet[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6},
                                             {5, 7}, {1, 2}, {5, 6}, {0, 4}, {1, 5}, {2, 6}, {3, 7},
                                             {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
                for (int c = 0; c < 19; ++c) {
                    const int x = sv[kNet[c][0]], y = sv[kNet[c][1]];
                    sv[kNet[c][0]] = min(x, y);
                    sv[kNet[c][1]] = max(x, y);
                }
                const int want = (n - 1) / 2;
                int res = -1;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (n > 0 && k == want) res = sv[k];
                o[i] = (int16_t)res;
            }
            __syncthreads();
            cur ^= 1;
        }
        // this thread's pixel of the tile
        const int lx = threadIdx.x % kPrepTX, ly = threadIdx.x / kPrepTX;
        const int x = bx * kPrepTX + lx, y = by * kPrepTY + ly;
        if (x < W && y < H) {
            const int p = y * W + x;
            const int d = buf[cur][(ly + F) * EW + lx + F];
            a.fuse.dinit[p] = (int16_t)d;
            borders_pixel<T>(a.brd, p, d);
        }
    }
}

// --- boundary-less search (Sec. 4.5): every pixel keeps the full range -------
struct FullArgs {
    gptr<int16_t> lo;
    gptr<int16_t> hi;
    int HW, N;
};

template <class Src>
__global__ __launch_bounds__(kThreads) void full_range_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const FullArgs& a = member(src, vb, b);
        const int p = (int)b * kThreads + threadIdx.x;
        if (p >= a.HW) continue;
        a.lo[p] = 0;
        a.hi[p] = (int16_t)(a.N - 1);
    }
}

// --- exclusive prefix sum of the range widths -> CSR offsets ----------------
// Two launches: per-tile totals, then per tile the sum of the totals before it
// (its base) and the scan of its own widths.
constexpr int kScanPerThread = 8;
constexpr int kScanTile = kThreads * kScanPerThread;

struct ScanArgs {
    gptr<const int16_t> lo;
    gptr<const int16_t> hi;
    gptr<int64_t> bsum;            // [nb]: tile totals
    gptr<int64_t> offsets;         // [HW + 1]
    int64_t HW;
    int nb;
};

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

template <class Src>
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(Src src) {
    __shared__ int64_t sh[kThreads];
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const ScanArgs& a = member(src, vb, b);
        const int64_t base = (int64_t)b * kScanTile;
        int64_t s = 0;
        for (int i = 0; i < kScanPerThread; ++i) {
            const int64_t p = base + (int64_t)i * kThreads + threadIdx.x;
            if (p < a.HW) s += (int64_t)(a.hi[p] - a.lo[p] + 1);
        }
        int64_t total;
        block_exclusive_scan(s, sh, total);
        if (threadIdx.x == 0) a.bsum[b] = total;
    }
}

template <class Src>
__global__ __launch_bounds__(kThreads) void scan_apply_kernel(Src src) {
    __shared__ int64_t sh[kThreads];
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const ScanArgs& a = member(src, vb, b);
        // the tile's base: the sum of the totals of the tiles before it (a tile
        // count of HW / 2048, so each thread adds a few)
        int64_t pre = 0;
        for (int i = threadIdx.x; i < (int)b; i += kThreads) pre += a.bsum[i];
        int64_t tile_base;
        block_exclusive_scan(pre, sh, tile_base);
        // each thread owns kScanPerThread consecutive pixels of the tile
        const int64_t base = (int64_t)b * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
        int w[kScanPerThread];
        int64_t s = 0;
        for (int i = 0; i < kScanPerThread; ++i) {
            const int64_t p = base + i;
            w[i] = p < a.HW ? a.hi[p] - a.lo[p] + 1 : 0;
            s += w[i];
        }
        int64_t total;
        int64_t run = tile_base + block_exclusive_scan(s, sh, total);
        for (int i = 0; i < kScanPerThread; ++i) {
            const int64_t p = base + i;
            if (p < a.HW) a.offsets[p] = run;
            run += w[i];
        }
        if ((int)b == a.nb - 1 && threadIdx.x == 0) a.offsets[a.HW] = tile_base + total;
    }
}

// --- WTA (Eq. 10) and the parabola sub-pixel step (Sec. 3.6) ----------------
struct WtaArgs {
    gptr<const void> csum;
    gptr<const int64_t> off;
    gptr<const int16_t> lo;
    gptr<const int16_t> hi;
    gptr<const float> hyp;
    gptr<int16_t> d_index;
    gptr<float> disp;
    int HW, N;
};

template <typename SumT>
__device__ __forceinline__ void wta_pixel(const WtaArgs& a, int p) {
    // bounds outside the documented 0 <= lo <= hi < N are clamped into it, so no
    // hypothesis outside [0, N) is read (the result is then unspecified)
    const int l = clampi(a.lo[p], 0, a.N - 1), h = clampi(a.hi[p], l, a.N - 1);
    const SumT* c = (const SumT*)a.csum + a.off[p] - l;     // c[k] for k in [l, h]
    const float* hyp = a.hyp;
    // in increasing k, strict <, so the lowest index wins ties; eight loads in
    // flight per round (indices past h re-read c[h] and are not compared)
    int best = l;
    uint32_t bv = c[l];
    for (int k0 = l + 1; k0 <= h; k0 += 8) {
        uint32_t x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = c[min(k0 + i, h)];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (k0 + i <= h && x[i] < bv) {
                bv = x[i];
                best = k0 + i;
            }
    }
    a.d_index[p] = (int16_t)best;
    float d = hyp[best];
    if (best - 1 >= l && best + 1 <= h && h - l >= 4) {
        const int64_t cm = c[best - 1], c0 = c[best], cp = c[best + 1];
        const float o = (float)(cm - cp) / (2.0f * (float)(cm + cp - 2 * c0));
        d = o >= 0.0f ? fmaf(o, hyp[best + 1] - hyp[best], hyp[best])
                      : fmaf(o, hyp[best] - hyp[best - 1], hyp[best]);
    }
    a.disp[p] = d;
}

template <class Src, typename SumT>
__global__ __launch_bounds__(kThreads) void wta_subpixel_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const WtaArgs& a = member(src, vb, b);
        const int p = (int)b * kThreads + threadIdx.x;
        if (p < a.HW) wta_pixel<SumT>(a, p);
    }
}

// --- 3x3 median, clamp-to-edge ----------------------------------------------
struct MedianArgs {
    gptr<const float> in;
    gptr<float> out;
    int H, W;
};

__device__ __forceinline__ void median_pixel(const MedianArgs& a, int p) {
    const int H = a.H, W = a.W;
    const int v = p / W, u = p - v * W;
    float w[9];
    int n = 0;
    for (int i = -1; i <= 1; ++i) {
        const int y = clampi(v + i, 0, H - 1);
        for (int j = -1; j <= 1; ++j) w[n++] = a.in[(size_t)y * W + clampi(u + j, 0, W - 1)];
    }
    // rank selection: the median has at most 4 values below it and at least 5 at or below
    float med = w[4];
#pragma unroll
    for (int x = 0; x < 9; ++x) {
        int below = 0, atmost = 0;
#pragma unroll
        for (int y = 0; y < 9; ++y) {
            below += w[y] < w[x];
            atmost += w[y] <= w[x];
        }
        if (below <= 4 && 4 < atmost) med = w[x];
    }
    a.out[p] = med;
}

template <class Src>
__global__ __launch_bounds__(kThreads) void median3_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const MedianArgs& a = member(src, vb, b);
        const int p = (int)b * kThreads + threadIdx.x;
        if (p < a.H * a.W) median_pixel(a, p);
    }
}

}  // namespace

size_t scan_scratch_bytes(int64_t HW) {
    const int64_t nb = (HW + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * sizeof(int64_t);
}

hipError_t stage_borders(Runner& r, const Jobs& jobs) {
    // light fields with at most kMaxPrepFill fill passes: one tile kernel; others:
    // fusion, the fill passes and the borders as separate launches
    std::vector<PrepArgs> prep[2];
    std::vector<uint32_t> prep_blocks[2];
    std::vector<FuseArgs> fuse;
    std::vector<uint32_t> fuse_blocks;
    std::vector<BordersArgs> brd[2];
    std::vector<uint32_t> brd_blocks[2];
    Jobs sep;
    int max_passes = 0;
    for (const Job* j : jobs) {
        const int HW = j->H * j->W;
        const int t = j->dtype == LF_U8 ? 0 : 1;
        const int sh = (j->S - 1) / 2, th = (j->T - 1) / 2;
        const size_t elem = j->dtype == LF_U8 ? 1 : 4;
        BordersArgs b{};
        b.dinit = j->dinit;
        b.ref = (const char*)j->views + ((size_t)th * j->S + sh) * j->C * j->H * j->pitch * elem;
        b.lo = j->lo;
        b.hi = j->hi;
        b.pitch = j->pitch;
        b.H = j->H;
        b.W = j->W;
        b.N = j->N;
        b.lambda = j->prm.lambda;
        b.lambda_far = j->prm.lambda_far;
        b.C = j->C;
        b.alpha = j->alpha;
        b.tau = j->prm.edge_tau;
        if (j->prm.fill_passes <= kMaxPrepFill) {
            PrepArgs pa{};
            pa.fuse = FuseArgs{j->maps, j->dinit, j->nv, HW, j->prm.phi};
            pa.brd = b;
            pa.fill = j->prm.fill_passes;
            pa.tx = (j->W + kPrepTX - 1) / kPrepTX;
            prep[t].push_back(pa);
            prep_blocks[t].push_back((uint32_t)pa.tx * ((j->H + kPrepTY - 1) / kPrepTY));
            continue;
        }
        sep.push_back(j);
        int16_t* buf[2] = {j->dinit, j->fill_tmp};
        // the passes ping-pong between the two buffers and end in dinit
        fuse.push_back(FuseArgs{j->maps, buf[j->prm.fill_passes % 2], j->nv, HW, j->prm.phi});
        fuse_blocks.push_back(blocks_for(HW));
        max_passes = std::max(max_passes, j->prm.fill_passes);
        brd[t].push_back(b);
        brd_blocks[t].push_back(blocks_for(HW));
    }
    hipError_t e = hipSuccess;
    if (!prep[0].empty() &&
        (e = launch(r, kStBorders, prep_kernel<Single<PrepArgs>, uint8_t>,
                    prep_kernel<Group<PrepArgs>, uint8_t>, prep[0], prep_blocks[0],
                    kThreads)) != hipSuccess)
        return e;
    if (!prep[1].empty() &&
        (e = launch(r, kStBorders, prep_kernel<Single<PrepArgs>, float>,
                    prep_kernel<Group<PrepArgs>, float>, prep[1], prep_blocks[1],
                    kThreads)) != hipSuccess)
        return e;
    if (sep.empty()) return hipSuccess;
    e = launch(r, kStBorders, fuse_kernel<Single<FuseArgs>>, fuse_kernel<Group<FuseArgs>>, fuse,
               fuse_blocks, kThreads);
    if (e != hipSuccess) return e;
    for (int f = 0; f < max_passes; ++f) {
        std::vector<FillArgs> fill;
        std::vector<uint32_t> fill_blocks;
        for (const Job* j : sep) {
            if (f >= j->prm.fill_passes) continue;
            int16_t* buf[2] = {j->dinit, j->fill_tmp};
            const int cur = (j->prm.fill_passes + f) % 2;
            fill.push_back(FillArgs{buf[cur], buf[cur ^ 1], j->H, j->W});
            fill_blocks.push_back(blocks_for((int64_t)j->H * j->W));
        }
        e = launch(r, kStBorders, fill_kernel<Single<FillArgs>>, fill_kernel<Group<FillArgs>>,
                   fill, fill_blocks, kThreads);
        if (e != hipSuccess) return e;
    }
    if (!brd[0].empty()) {
        e = launch(r, kStBorders, borders_kernel<Single<BordersArgs>, uint8_t>,
                   borders_kernel<Group<BordersArgs>, uint8_t>, brd[0], brd_blocks[0], kThreads);
        if (e != hipSuccess) return e;
    }
    if (!brd[1].empty())
        e = launch(r, kStBorders, borders_kernel<Single<BordersArgs>, float>,
                   borders_kernel<Group<BordersArgs>, float>, brd[1], brd_blocks[1], kThreads);
    return e;
}

hipError_t stage_full_range(Runner& r, const Jobs& jobs) {
    std::vector<FullArgs> args;
    std::vector<uint32_t> blocks;
    for (const Job* j : jobs) {
        args.push_back(FullArgs{j->lo, j->hi, j->H * j->W, j->N});
        blocks.push_back(blocks_for((int64_t)j->H * j->W));
    }
    return launch(r, kStBorders, full_range_kernel<Single<FullArgs>>,
                  full_range_kernel<Group<FullArgs>>, args, blocks, kThreads);
}

hipError_t stage_offsets(Runner& r, const Jobs& jobs) {
    std::vector<ScanArgs> args;
    std::vector<uint32_t> tiles;
    for (const Job* j : jobs) {
        const int64_t HW = (int64_t)j->H * j->W;
        ScanArgs a{};
        a.lo = j->lo;
        a.hi = j->hi;
        a.bsum = (int64_t*)j->scan;
        a.offsets = j->offsets;
        a.HW = HW;
        a.nb = (int)((HW + kScanTile - 1) / kScanTile);
        args.push_back(a);
        tiles.push_back((uint32_t)a.nb);
    }
    hipError_t e = launch(r, kStOffsets, scan_reduce_kernel<Single<ScanArgs>>,
                          scan_reduce_kernel<Group<ScanArgs>>, args, tiles, kThreads);
    if (e != hipSuccess) return e;
    return launch(r, kStOffsets, scan_apply_kernel<Single<ScanArgs>>,
                  scan_apply_kernel<Group<ScanArgs>>, args, tiles, kThreads);
}

hipError_t stage_wta(Runner& r, const Jobs& jobs) {
    std::vector<WtaArgs> wta[2];
    std::vector<uint32_t> wta_blocks[2];
    std::vector<MedianArgs> med;
    std::vector<uint32_t> med_blocks;
    for (const Job* j : jobs) {
        const int HW = j->H * j->W;
        const bool median = j->prm.median == 3;
        WtaArgs a{};
        a.csum = j->csum;
        a.off = j->offsets;
        a.lo = j->lo;
        a.hi = j->hi;
        a.hyp = j->hyp;
        a.d_index = j->d_index;
        a.disp = median ? j->pre_median : j->disparity;
        a.HW = HW;
        a.N = j->N;
        const int sb = j->prm.sum_bits == 16 ? 0 : 1;
        wta[sb].push_back(a);
        wta_blocks[sb].push_back(blocks_for(HW));
        if (median) {
            med.push_back(MedianArgs{j->pre_median, j->disparity, j->H, j->W});
            med_blocks.push_back(blocks_for(HW));
        }
    }
    hipError_t e = hipSuccess;
    if (!wta[0].empty()) {
        e = launch(r, kStWta, wta_subpixel_kernel<Single<WtaArgs>, uint16_t>,
                   wta_subpixel_kernel<Group<WtaArgs>, uint16_t>, wta[0], wta_blocks[0], kThreads);
        if (e != hipSuccess) return e;
    }
    if (!wta[1].empty()) {
        e = launch(r, kStWta, wta_subpixel_kernel<Single<WtaArgs>, uint32_t>,
                   wta_subpixel_kernel<Group<WtaArgs>, uint32_t>, wta[1], wta_blocks[1], kThreads);
        if (e != hipSuccess) return e;
    }
    if (!med.empty())
        e = launch(r, kStWta, median3_kernel<Single<MedianArgs>>, median3_kernel<Group<MedianArgs>>,
                   med, med_blocks, kThreads);
    return e;
}

}  // namespace lf
