// Bounded matching cost over all views, Sec. 3.5: Eq. (12) (l2 of the
// bilinearly shifted views) and Eq. (15) (Census Hamming at the nearest shift).
//
// Work is flattened over the cells of the CSR volume so that pixels whose range
// is the full hypothesis set and pixels with a 2*lambda+1 window share the
// machine evenly; a cell finds its pixel by binary search over offsets staged in
// LDS.  Consecutive threads handle consecutive hypotheses of one pixel and then
// the next pixel of the row, so the bilinear taps of a view are read from a
// narrow band of two rows (L1/L2 resident) and the cost writes are coalesced.
//
// The view loop runs t outer, s inner, float32, with the shift of each view and
// hypothesis rounded once: this is the precision the quantised integer cost is
// decided in.  The reference view contributes exactly +0 and is skipped.
#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kPix = 64;        // pixels per workgroup (Census kind)
constexpr int kThreads = 256;

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
// l2 cost, Eq. (12).  Work is dealt in equal slices of cells: slice i is the
// cells [i*chunk, (i+1)*chunk) of the CSR volume, whatever pixels they belong
// to, so pixels with the full hypothesis range and pixels with a 2*lambda+1
// window cost the same per cell and no workgroup is a straggler.  The number of
// slices is only known on the device (the last offset), so a light field gets
// nblk workgroups sized for its worst case, and workgroup b walks the slices
// b, b + nblk, ... that exist.  The first pixel of a slice is found by binary
// search over the offsets; the offsets and lower bounds of the slice's pixels
// are staged in LDS, and each cell finds its pixel there.  Consecutive threads
// take consecutive cells (consecutive hypotheses of a pixel, then the next
// pixel).
//
// Per view the two taps of a bilinear row, (x0, x0+1), are fetched by one 8-byte
// load (the view pointer is only 4-byte aligned, which global loads allow):
// that halves the gather instructions, whose issue rate -- not bytes -- bounds
// this kernel.  At the image edges a tap is clamped; the pair then starts at
// min(x_a, W-2) and each tap picks its element of the pair.
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

// Pixels per group of the grayscale float l2 cost (see l2_slices).
constexpr int kGroup = 3;

// Views with a replicated edge: padded (y', x') holds the view at
// (clamp(y' - 1), clamp(x' - kGroup)), y' < H + 2, x' < W + 2 kGroup (one row
// above and below, kGroup columns left and right).  With it, the two clamped
// taps of a bilinear row, (clamp(X), clamp(X+1)), are always the two consecutive
// elements starting at clamp(X, -1, W-1) + kGroup -- one 8-byte load, no edge
// cases, and the same values (so the same float32 sums) as clamping each tap;
// and the taps of the pixels g = 1 .. kGroup-1 to the right, (clamp(X+g),
// clamp(X+g+1)), are always elements g, g+1 of the kGroup+1 starting at
// clamp(X, -kGroup, W-1) + kGroup (X outside that range reads replicas).
constexpr int kPadL = kGroup, kPadT = 1;
static_assert(kPadW == 2 * kGroup && kPadH == 2, "view copy margins");

struct PadArgs {
    gptr<const void> src;          // [planes][H][pitch] (a view is C planes)
    gptr<void> dst;                // [planes][H + 2][W + 2 kGroup]
    int H, W, pitch;
};

// A workgroup copies kPadRows padded rows of one plane: block b is rows
// kPadRows * (b % g) .. of plane b / g (g row groups per plane).  Each thread
// loads its elements of all the rows (3 x kPadRows per 768 columns) before it
// stores them, so that many loads are in flight.
constexpr int kPadRows = 4;

template <class Src, typename T>
__global__ __launch_bounds__(kThreads) void pad_views_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const PadArgs& a = member(src, vb, b);
        const int Hp = a.H + kPadH, Wp = a.W + kPadW;
        const int g = (Hp + kPadRows - 1) / kPadRows;
        const int z = (int)(b / (uint32_t)g);
        const int y0 = ((int)b - z * g) * kPadRows;
        for (int xb = 0; xb < Wp; xb += 3 * kThreads) {
            T v[kPadRows][3];
#pragma unroll
            for (int r = 0; r < kPadRows; ++r) {
                const T* __restrict__ row =
                    (const T*)a.src +
                    ((size_t)z * a.H + clampi(y0 + r - kPadT, 0, a.H - 1)) * a.pitch;
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const int x = xb + e * kThreads + (int)threadIdx.x;
                    v[r][e] = row[clampi(x - kPadL, 0, a.W - 1)];
                }
            }
#pragma unroll
            for (int r = 0; r < kPadRows; ++r) {
                if (y0 + r >= Hp) break;
                T* __restrict__ out = (T*)a.dst + ((size_t)z * Hp + y0 + r) * Wp;
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const int x = xb + e * kThreads + (int)threadIdx.x;
                    if (x < Wp) out[x] = v[r][e];
                }
            }
        }
    }
}

struct L2Args {
    gptr<const void> views;        // padded: [T][S][C][H + 2][W + 2 kGroup]
    gptr<const float> hyp;
    gptr<const int16_t> lo;
    gptr<const int64_t> off;       // [H*W + 1]
    gptr<uint16_t> cost;
    gptr<float> cost_f32;          // nullable
    int64_t cap_cells;
    int S, T, H, W, N;
    float alpha, cap;
    uint32_t nblk;            // workgroups of this light field
};

// kGroup + 1 consecutive elements of a padded float view row, one load.
struct Row {
    float e[kGroup + 1];
};
__device__ __forceinline__ Row ld_row(const float* p) {
    Row r;
    __builtin_memcpy(&r, p, sizeof(Row));
    return r;
}

// Block-wide exclusive prefix sum of cnt(i) over i in [0, np) into s_pre[0..np]
// (s_pre[np] = the total); thread t owns the E consecutive entries from t*E.
template <class Cnt>
__device__ __forceinline__ void block_prefix(int np, Cnt cnt, int* s_pre, int* s_tmp) {
    const int E = (np + kThreads - 1) / kThreads;
    int local = 0;
    for (int e = 0; e < E; ++e) {
        const int i = threadIdx.x * E + e;
        if (i < np) local += cnt(i);
    }
    s_tmp[threadIdx.x] = local;
    __syncthreads();
    if (threadIdx.x < 64) {                           // wave 0 scans the 256 sums
        const int l = threadIdx.x;
        const int v0 = s_tmp[4 * l], v1 = s_tmp[4 * l + 1], v2 = s_tmp[4 * l + 2],
                  v3 = s_tmp[4 * l + 3];
        const int own = v0 + v1 + v2 + v3;
        int inc = own;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int n = __shfl_up(inc, o);
            if (l >= o) inc += n;
        }
        const int ex = inc - own;
        s_tmp[4 * l] = ex;
        s_tmp[4 * l + 1] = ex + v0;
        s_tmp[4 * l + 2] = ex + v0 + v1;
        s_tmp[4 * l + 3] = ex + v0 + v1 + v2;
        if (l == 63) s_pre[np] = inc;
    }
    __syncthreads();
    int run = s_tmp[threadIdx.x];
    for (int e = 0; e < E; ++e) {
        const int i = threadIdx.x * E + e;
        if (i < np) {
            s_pre[i] = run;
            run += cnt(i);
        }
    }
    __syncthreads();
}

template <typename T, int CPT, bool Walk, int C>
__device__ __forceinline__ void l2_slices(const L2Args& a, uint32_t b, int64_t* s_off, int* s_lo,
                                          int* s_p, int* s_pre, int* s_tmp) {
    // float grayscale views: the cells of two horizontally adjacent pixels at one
    // hypothesis share their loads (see below)
    constexpr bool kPairs = sizeof(T) == 4 && C == 1;
    constexpr int kChunk = kThreads * CPT;
    const int S = a.S, T_ = a.T, H = a.H, W = a.W, N = a.N;
    const int Wp = W + kPadW;
    const int16_t* __restrict__ lo = a.lo;
    const int64_t* __restrict__ off = a.off;
    const int HW = H * W;
    const int64_t total = min(off[HW], a.cap_cells);
    const int sh = (S - 1) / 2, th = (T_ - 1) / 2;
    const uint32_t vstride = (uint32_t)(H + kPadH) * Wp;
    const T* __restrict__ views = (const T*)a.views;
    const T* __restrict__ refv = views + ((size_t)th * S + sh) * C * vstride;

    auto store = [&](int64_t c, float acc) {
        const float q = rintf(a.alpha * acc);
        a.cost[c] = (uint16_t)(q > a.cap ? a.cap : q);
        if (a.cost_f32) a.cost_f32[c] = acc;
    };

    // Eq. (12) for one cell: pixel (u, v), hypothesis d, over the views t outer,
    // s inner.  One view of row t takes taps at horizontal fraction fx from the
    // rows rt and rt + Wp.  Two cases skip taps that are weighted by an exact 0,
    // since fma(0, b - a, a) is a exactly: the reference row of views (t = t_hat,
    // flat: fy = 0, no bottom taps) and the reference column (s = s_hat, col:
    // fx = 0, only the left tap of each row).  Each case is its own branch-free
    // copy of the loop body.
    auto cell = [&](int u, int v, float d) -> float {
        float ref[C];
#pragma unroll
        for (int c = 0; c < C; ++c)
            ref[c] = ld(refv + (uint32_t)c * vstride + (uint32_t)(v + kPadT) * Wp + u + kPadL);
        float acc = 0.0f;
        auto view = [&](const T* __restrict__ vt, uint32_t rt, float fy, int s, bool flat,
                        bool col) {
            const float shx = (float)(sh - s) * d;
            const float x0 = floorf(shx);
            const float fx = shx - x0;
            const uint32_t o = rt + (uint32_t)(clampi(u + (int)x0, -1, W - 1) + kPadL);
            float sq = 0.0f, dist = 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T* __restrict__ vs = vt + (uint32_t)(s * C + c) * vstride;
                float tv, val;
                if (col) {
                    tv = ld(vs + o);
                    val = flat ? tv : fmaf(fy, ld(vs + o + Wp) - tv, tv);
                } else {
                    const Pair<T> top = ld_pair(vs + o);
                    tv = fmaf(fx, top.hi - top.lo, top.lo);
                    val = tv;
                    if (!flat) {
                        const Pair<T> bot = ld_pair(vs + o + Wp);
                        const float bv = fmaf(fx, bot.hi - bot.lo, bot.lo);
                        val = fmaf(fy, bv - tv, tv);
                    }
                }
                const float dl = ref[c] - val;
                dist = fabsf(dl);
                sq = c == 0 ? dl * dl : fmaf(dl, dl, sq);   // colour: l2 norm
            }
            acc = acc + (C == 1 ? dist : sqrtf(sq));
        };
        // s ascending; the reference view itself adds exactly +0 and is skipped
        auto view_row = [&](const T* __restrict__ vt, uint32_t rt, float fy, bool flat) {
            for (int s = 0; s < sh; ++s) view(vt, rt, fy, s, flat, false);
            if (!flat) view(vt, rt, fy, sh, false, true);
            for (int s = sh + 1; s < S; ++s) view(vt, rt, fy, s, flat, false);
        };
        for (int t = 0; t < T_; ++t) {
            const float shy = (float)(th - t) * d;
            const float y0 = floorf(shy);
            const float fy = shy - y0;
            // top tap row in padded coordinates; the bottom one follows it
            const uint32_t rt = (uint32_t)(clampi(v + (int)y0, -1, H - 1) + kPadT) * Wp;
            const T* __restrict__ vt = views + (size_t)t * S * C * vstride;
            if (t == th) view_row(vt, rt, fy, true);
            else view_row(vt, rt, fy, false);
        }
        return acc;
    };

    // Eq. (12) for the kGroup pixels (u + g, v) at one hypothesis d, with the
    // arithmetic of cell() for each.  The shift of a view is the same for all of
    // them, so pixel g's taps are pixel 0's moved by g elements: one load of
    // kGroup + 1 elements per tap row serves the group (kGroup elements for the
    // reference column of views, where only each pixel's left tap counts).
    auto group = [&](int u, int v, float d, float (&acc)[kGroup]) {
        const float* __restrict__ fv = (const float*)views;
        const float* __restrict__ rp =
            fv + ((size_t)th * S + sh) * vstride + (uint32_t)(v + kPadT) * Wp + u + kPadL;
        float ref[kGroup];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
            ref[g] = rp[g];
            acc[g] = 0.0f;
        }
        auto view = [&](const float* __restrict__ vt, uint32_t rt, float fy, int s, bool flat,
                        bool col) {
            const float shx = (float)(sh - s) * d;
            const float x0 = floorf(shx);
            const float fx = shx - x0;
            const float* __restrict__ pv = vt + (uint32_t)s * vstride + rt +
                                           (uint32_t)(clampi(u + (int)x0, -kPadL, W - 1) + kPadL);
            float val[kGroup];
            if (col) {                            // fx = 0: the left taps only
                float top[kGroup];
                __builtin_memcpy(&top, pv, sizeof(top));
#pragma unroll
                for (int g = 0; g < kGroup; ++g) val[g] = top[g];
                if (!flat) {
                    float bot[kGroup];
                    __builtin_memcpy(&bot, pv + Wp, sizeof(bot));
#pragma unroll
                    for (int g = 0; g < kGroup; ++g) val[g] = fmaf(fy, bot[g] - val[g], val[g]);
                }
            } else {
                const Row top = ld_row(pv);
#pragma unroll
                for (int g = 0; g < kGroup; ++g)
                    val[g] = fmaf(fx, top.e[g + 1] - top.e[g], top.e[g]);
                if (!flat) {
                    const Row bot = ld_row(pv + Wp);
#pragma unroll
                    for (int g = 0; g < kGroup; ++g) {
                        const float bv = fmaf(fx, bot.e[g + 1] - bot.e[g], bot.e[g]);
                        val[g] = fmaf(fy, bv - val[g], val[g]);
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < kGroup; ++g) acc[g] = acc[g] + fabsf(ref[g] - val[g]);
        };
        auto view_row = [&](const float* __restrict__ vt, uint32_t rt, float fy, bool flat) {
            for (int s = 0; s < sh; ++s) view(vt, rt, fy, s, flat, false);
            if (!flat) view(vt, rt, fy, sh, false, true);
            for (int s = sh + 1; s < S; ++s) view(vt, rt, fy, s, flat, false);
        };
        for (int t = 0; t < T_; ++t) {
            const float shy = (float)(th - t) * d;
            const float y0 = floorf(shy);
            const float fy = shy - y0;
            const uint32_t rt = (uint32_t)(clampi(v + (int)y0, -1, H - 1) + kPadT) * Wp;
            const float* __restrict__ vt = fv + (size_t)t * S * vstride;
            if (t == th) view_row(vt, rt, fy, true);
            else view_row(vt, rt, fy, false);
        }
    };

    for (int64_t slice = b; slice * kChunk < total; slice += a.nblk) {   // uniform
        const int64_t c0 = slice * kChunk;
        const int64_t c1 = min(c0 + kChunk, total);
        if constexpr (Walk) __syncthreads();      // LDS of the previous slice is read
        if (threadIdx.x == 0) {
            int x = 0, y = HW;                    // off[x] <= c0 < off[y]
            while (y - x > 1) {
                const int mid = (x + y) >> 1;
                if (off[mid] <= c0) x = mid; else y = mid;
            }
            s_p[0] = x;
            s_p[1] = min(kChunk, HW - x);
        }
        __syncthreads();
        const int p0 = s_p[0], npx = s_p[1];
        for (int i = threadIdx.x; i <= npx; i += kThreads) {
            s_off[i] = off[p0 + i];
            if (i < npx) s_lo[i] = lo[p0 + i];
        }
        __syncthreads();
        int np;                                   // pixels that own cells of the slice
        {
            int x = 0, y = npx;                   // largest i with s_off[i] <= c1 - 1
            while (y - x > 1) {
                const int mid = (x + y) >> 1;
                if (s_off[mid] <= c1 - 1) x = mid; else y = mid;
            }
            np = x + 1;
        }

        if constexpr (kPairs) {
            // Groups of the slice's pixels: a pixel at u = 0 mod kGroup (or the
            // slice's first pixel) with the following pixels of its row up to the
            // next such u that are in the slice.  A group's items are the
            // hypotheses k of the hull of its pixels' slice cells; an item
            // computes the cells (p + g, k) of the group that exist.
            auto first = [&](int i) { return max(s_off[i], c0); };       // slice cells of
            auto last = [&](int i) { return min(s_off[i + 1], c1) - 1; }; // pixel i
            auto kfirst = [&](int i) { return s_lo[i] + (int)(first(i) - s_off[i]); };
            auto klast = [&](int i) { return s_lo[i] + (int)(last(i) - s_off[i]); };
            auto ucol = [&](int i) { return (p0 + i) % W; };
            auto leads = [&](int i) { return i == 0 || ucol(i) % kGroup == 0; };
            auto members = [&](int i) {           // pixels of the group led by pixel i
                const int u = ucol(i);
                return min(min(kGroup - u % kGroup, np - i), W - u);
            };
            // hull [kl, kh] of the group led by pixel i (a pixel whose range is
            // empty -- possible only for bounds given with hi < lo -- adds nothing)
            auto hull = [&](int i, int n, int& kl, int& kh) {
                kl = INT_MAX;
                kh = INT_MIN;
                for (int g = 0; g < n; ++g)
                    if (first(i + g) <= last(i + g)) {
                        kl = min(kl, kfirst(i + g));
                        kh = max(kh, klast(i + g));
                    }
                return kl <= kh;
            };
            auto count = [&](int i) {
                int kl, kh;
                return leads(i) && hull(i, members(i), kl, kh) ? kh - kl + 1 : 0;
            };
            block_prefix(np, count, s_pre, s_tmp);
            const int nitems = s_pre[np];
            for (int j = threadIdx.x; j < nitems; j += kThreads) {
                int x = 0, y = np;                // largest i with s_pre[i] <= j
                while (y - x > 1) {
                    const int mid = (x + y) >> 1;
                    if (s_pre[mid] <= j) x = mid; else y = mid;
                }
                const int i = x;
                const int n = members(i);
                int kl, kh;
                hull(i, n, kl, kh);
                const int k = kl + (j - s_pre[i]);
                bool has[kGroup], any = false;
#pragma unroll
                for (int g = 0; g < kGroup; ++g) {
                    has[g] = g < n && k >= kfirst(i + g) && k <= klast(i + g) &&
                             (unsigned)k < (unsigned)N;
                    any |= has[g];
                }
                if (!any) continue;               // a gap of the hull, or a range
                const int p = p0 + i;             // outside [0, N)
                const int v = p / W, u = p - v * W;
                float acc[kGroup];
                group(u, v, a.hyp[k], acc);
#pragma unroll
                for (int g = 0; g < kGroup; ++g)
                    if (has[g]) store(s_off[i + g] + (k - s_lo[i + g]), acc[g]);
            }
        } else {
            for (int r = 0; r < CPT; ++r) {
                const int64_t c = c0 + threadIdx.x + (int64_t)r * kThreads;
                if (c >= c1) break;
                const int i = find_pixel(s_off, np, c);
                const int p = p0 + i;
                const int v = p / W, u = p - v * W;
                const int k = s_lo[i] + (int)(c - s_off[i]);
                if ((unsigned)k >= (unsigned)N) continue;      // only for ranges outside [0, N)
                store(c, cell(u, v, a.hyp[k]));
            }
        }
        if constexpr (!Walk) break;               // one slice per workgroup
    }
}

template <class Src, typename T, int CPT, bool Walk, int C>
__global__ __launch_bounds__(kThreads) void cost_l2_kernel(Src src) {
    constexpr bool kPairs = sizeof(T) == 4 && C == 1;
    __shared__ int64_t s_off[kThreads * CPT + 1];
    __shared__ int s_lo[kThreads * CPT];
    __shared__ int s_p[2];
    __shared__ int s_pre[kPairs ? kThreads * CPT + 1 : 1];
    __shared__ int s_tmp[kPairs ? kThreads : 1];
    uint32_t b;
    const L2Args& a = member(src, blockIdx.x, b);
    l2_slices<T, CPT, Walk, C>(a, b, s_off, s_lo, s_p, s_pre, s_tmp);
}

// ---------------------------------------------------------------------------
// Census kind, Eq. (15): 64 pixels per workgroup, their cells strided over the
// threads.
struct CensusAllArgs {
    gptr<const uint64_t> census;   // [S*T][C][H*W]
    gptr<const float> hyp;
    gptr<const int16_t> lo;
    gptr<const int64_t> off;
    gptr<uint16_t> cost;
    gptr<float> cost_f32;
    int64_t cap_cells;
    int S, T, C, H, W, N;
    uint32_t cap;
};

template <class Src>
__global__ __launch_bounds__(kThreads) void cost_census_all_kernel(Src src) {
    __shared__ int64_t s_off[kPix + 1];
    __shared__ int s_lo[kPix];
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const CensusAllArgs& a = member(src, vb, b);
        const int S = a.S, T_ = a.T, H = a.H, W = a.W, N = a.N;
        const int HW = H * W;
        const int p0 = (int)b * kPix;
        const int np = min(kPix, HW - p0);
        __syncthreads();
        for (int i = threadIdx.x; i <= np; i += kThreads) {
            s_off[i] = a.off[p0 + i];
            if (i < np) s_lo[i] = a.lo[p0 + i];
        }
        __syncthreads();
        const int sh = (S - 1) / 2, th = (T_ - 1) / 2;
        const int C = a.C;
        const uint64_t* __restrict__ census = a.census;
        const uint64_t* __restrict__ cref = census + ((size_t)th * S + sh) * C * HW;
        for (int64_t c = s_off[0] + threadIdx.x; c < s_off[np]; c += kThreads) {
            if (c >= a.cap_cells) break;
            const int i = find_pixel(s_off, np, c);
            const int p = p0 + i;
            const int v = p / W, u = p - v * W;
            const int k = s_lo[i] + (int)(c - s_off[i]);
            if ((unsigned)k >= (unsigned)N) continue;
            const float d = a.hyp[k];
            uint32_t acc = 0;
            for (int t = 0; t < T_; ++t) {
                const int y = clampi(v + (int)rintf((float)(th - t) * d), 0, H - 1);
                for (int s = 0; s < S; ++s) {
                    const int x = clampi(u + (int)rintf((float)(sh - s) * d), 0, W - 1);
                    for (int c = 0; c < C; ++c)             // colour: summed per channel
                        acc += (uint32_t)__popcll(
                            cref[(size_t)c * HW + p] ^
                            census[(((size_t)t * S + s) * C + c) * HW + (size_t)y * W + x]);
                }
            }
            a.cost[c] = (uint16_t)min(acc, a.cap);
            if (a.cost_f32) a.cost_f32[c] = (float)acc;
        }
    }
}

template <typename T, bool Walk, int C>
hipError_t l2_variant(Runner& r, const std::vector<L2Args>& args,
                      const std::vector<uint32_t>& blocks) {
    switch (r.tune.cost_cpt) {
        case 2:
            return launch(r, kStCost, cost_l2_kernel<Single<L2Args>, T, 2, Walk, C>,
                          cost_l2_kernel<Group<L2Args>, T, 2, Walk, C>, args, blocks, kThreads);
        case 8:
            return launch(r, kStCost, cost_l2_kernel<Single<L2Args>, T, 8, Walk, C>,
                          cost_l2_kernel<Group<L2Args>, T, 8, Walk, C>, args, blocks, kThreads);
        default:
            return launch(r, kStCost, cost_l2_kernel<Single<L2Args>, T, 4, Walk, C>,
                          cost_l2_kernel<Group<L2Args>, T, 4, Walk, C>, args, blocks, kThreads);
    }
}

template <typename T, int C>
hipError_t l2_walk(Runner& r, const std::vector<L2Args>& args,
                   const std::vector<uint32_t>& blocks) {
    return r.tune.cost_stride > 1 ? l2_variant<T, true, C>(r, args, blocks)
                                  : l2_variant<T, false, C>(r, args, blocks);
}

}  // namespace

hipError_t stage_cost_inputs(Runner& r, const Jobs& jobs) {
    // l2 cost: the edge-replicated copy of every view plane; Eq. (15) cost: the
    // Census strings of every view
    std::vector<PadArgs> pads[2];
    std::vector<uint32_t> pad_blocks[2];
    Jobs census_jobs;
    for (const Job* j : jobs) {
        if (j->prm.cost_kind != LF_COST_L2) {
            census_jobs.push_back(j);
            continue;
        }
        PadArgs pa{};
        pa.src = j->views;
        pa.dst = j->padded;
        pa.H = j->H;
        pa.W = j->W;
        pa.pitch = j->pitch;
        pads[j->dtype == LF_U8 ? 0 : 1].push_back(pa);
        pad_blocks[j->dtype == LF_U8 ? 0 : 1].push_back(
            (uint32_t)((j->H + kPadH + kPadRows - 1) / kPadRows) * j->S * j->T * j->C);
    }
    hipError_t e = hipSuccess;
    if (!pads[0].empty() &&
        (e = launch(r, kStCostInputs, pad_views_kernel<Single<PadArgs>, uint8_t>,
                    pad_views_kernel<Group<PadArgs>, uint8_t>, pads[0], pad_blocks[0],
                    kThreads)) != hipSuccess)
        return e;
    if (!pads[1].empty() &&
        (e = launch(r, kStCostInputs, pad_views_kernel<Single<PadArgs>, float>,
                    pad_views_kernel<Group<PadArgs>, float>, pads[1], pad_blocks[1],
                    kThreads)) != hipSuccess)
        return e;
    if (!census_jobs.empty()) e = stage_census(r, census_jobs, true);
    return e;
}

hipError_t stage_cost(Runner& r, const Jobs& jobs) {
    std::vector<L2Args> l2[2][2];                  // [u8/f32][gray/colour]
    std::vector<uint32_t> l2_blocks[2][2];
    std::vector<CensusAllArgs> ca;
    std::vector<uint32_t> ca_blocks;
    const int cpt = r.tune.cost_cpt == 2 || r.tune.cost_cpt == 8 ? r.tune.cost_cpt : 4;
    const int stride = std::max(1, r.tune.cost_stride);
    for (const Job* j : jobs) {
        const int64_t HW = (int64_t)j->H * j->W;
        if (j->prm.cost_kind == LF_COST_L2) {
            L2Args a{};
            a.views = j->padded;
            a.hyp = j->hyp;
            a.lo = j->lo;
            a.off = j->offsets;
            a.cost = j->cost;
            a.cost_f32 = j->cost_f32;
            a.cap_cells = j->cap_cells;
            a.S = j->S;
            a.T = j->T;
            a.H = j->H;
            a.W = j->W;
            a.N = j->N;
            a.alpha = j->alpha;
            a.cap = (float)j->cap;
            // worst-case slices; those past the device-side cell count are skipped
            const int64_t slices = (HW * j->N + kThreads * cpt - 1) / (kThreads * cpt);
            a.nblk = (uint32_t)std::max<int64_t>(1, (slices + stride - 1) / stride);
            const int t = j->dtype == LF_U8 ? 0 : 1, col = j->C == 3 ? 1 : 0;
            l2[t][col].push_back(a);
            l2_blocks[t][col].push_back(a.nblk);
        } else {
            CensusAllArgs a{};
            a.census = j->census_all;
            a.hyp = j->hyp;
            a.lo = j->lo;
            a.off = j->offsets;
            a.cost = j->cost;
            a.cost_f32 = j->cost_f32;
            a.cap_cells = j->cap_cells;
            a.S = j->S;
            a.T = j->T;
            a.C = j->C;
            a.H = j->H;
            a.W = j->W;
            a.N = j->N;
            a.cap = (uint32_t)j->cap;
            ca.push_back(a);
            ca_blocks.push_back((uint32_t)((HW + kPix - 1) / kPix));
        }
    }
    hipError_t e = hipSuccess;
    if (!l2[0][0].empty() && (e = l2_walk<uint8_t, 1>(r, l2[0][0], l2_blocks[0][0])) != hipSuccess)
        return e;
    if (!l2[1][0].empty() && (e = l2_walk<float, 1>(r, l2[1][0], l2_blocks[1][0])) != hipSuccess)
        return e;
    if (!l2[0][1].empty() && (e = l2_walk<uint8_t, 3>(r, l2[0][1], l2_blocks[0][1])) != hipSuccess)
        return e;
    if (!l2[1][1].empty() && (e = l2_walk<float, 3>(r, l2[1][1], l2_blocks[1][1])) != hipSuccess)
        return e;
    if (!ca.empty())
        e = launch(r, kStCost, cost_census_all_kernel<Single<CensusAllArgs>>,
                   cost_census_all_kernel<Group<CensusAllArgs>>, ca, ca_blocks, kThreads);
    return e;
}

}  // namespace lf
