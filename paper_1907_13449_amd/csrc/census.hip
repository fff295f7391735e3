// Census transform, Sec. 3.2 Eq. (2)-(3), from LDS-staged tiles.
//
// A 256-thread workgroup owns a 32 x 8 pixel tile.  It stages the tile plus the
// window halo (clamp-to-edge) into LDS once, as float, with coalesced row loads,
// then each thread compares its centre with the win_h*win_w - 1 neighbours in
// row-major order (centre skipped), bit n = [centre > neighbour n] -- or, for a
// sparse window, with the listed neighbours, whose positions in the window are
// read by every lane from the launch record.
#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kBX = 32, kBY = 8;

// Up to kMaxBatchImages images of one size; image z starts at base + off[z]
// elements, or at base + z * stride when n > kMaxBatchImages.
struct CensusArgs {
    gptr<const void> base;
    int64_t off[kMaxBatchImages];
    int64_t stride;
    int n;
    int H, W, pitch, win_h, win_w;
    int bx, by;               // tiles along x and y
    gptr<uint64_t> out;            // [n][H*W]
    int ntap;                 // sparse window: neighbours listed (0: dense window)
    uint8_t tap[LF_MAX_CENSUS_BITS];    // neighbour n: row (dy + win_h/2) in bits 0-3,
                                        // column (dx + win_w/2) in bits 4-7
};

// The bit string of one pixel from its window in the LDS tile (win points at the
// window's top-left element, rows tw apart): bit n = [centre > neighbour n],
// neighbours in row-major order, centre skipped.
__device__ __forceinline__ uint64_t census_any(const float* win, int wh, int ww, int tw) {
    const int rh = wh / 2, rw = ww / 2;
    const float c = win[rh * tw + rw];
    uint64_t bits = 0;
    int n = 0;
    for (int i = 0; i < wh; ++i) {
        const float* row = win + i * tw;
        for (int j = 0; j < ww; ++j) {
            if (i == rh && j == rw) continue;
            bits |= (uint64_t)(c > row[j]) << n;
            ++n;
        }
    }
    return bits;
}

// The same for a window size known at compile time: every shift and LDS offset
// is a constant, and the two 32-bit halves are built separately.
template <int WH, int WW>
__device__ __forceinline__ uint64_t census_fixed(const float* win) {
    constexpr int tw = kBX + 2 * (WW / 2), rh = WH / 2, rw = WW / 2;
    const float c = win[rh * tw + rw];
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int i = 0, n = 0; i < WH; ++i)
#pragma unroll
        for (int j = 0; j < WW; ++j) {
            if (i == rh && j == rw) continue;
            const uint32_t bit = c > win[i * tw + j] ? 1u : 0u;
            if (n < 32) lo |= bit << n;
            else hi |= bit << (n - 32);
            ++n;
        }
    return ((uint64_t)hi << 32) | lo;
}

// The bit string over a listed neighbour set: bit n = [centre > neighbour n],
// neighbour n at window row tap & 15, column tap >> 4 (rows tw apart).  The list
// is uniform over the launch record: the taps and their offsets are scalar work.
template <class A>
__device__ __forceinline__ uint64_t census_listed(const float* win, const A& a, int tw,
                                                  int ctr) {
    const float c = win[ctr];
    const int n = a.ntap, n0 = n < 32 ? n : 32;
    uint32_t lo = 0, hi = 0;
    for (int i = 0; i < n0; ++i) {
        const int t = a.tap[i];
        lo |= (c > win[(t & 15) * tw + (t >> 4)] ? 1u : 0u) << i;
    }
    for (int i = 32; i < n; ++i) {
        const int t = a.tap[i];
        hi |= (c > win[(t & 15) * tw + (t >> 4)] ? 1u : 0u) << (i - 32);
    }
    return ((uint64_t)hi << 32) | lo;
}

template <typename T, int WH, int WW>
__device__ __forceinline__ void census_block(const CensusArgs& a, uint32_t b, float* tile) {
    const int per = a.bx * a.by;
    const int z = (int)b / per;
    const int rem = (int)b - z * per;
    const int by = rem / a.bx, bx = rem - by * a.bx;
    const int H = a.H, W = a.W;
    const int64_t off = a.n > kMaxBatchImages ? (int64_t)z * a.stride : a.off[z];
    const T* __restrict__ img = (const T*)(a.base) + off;
    uint64_t* __restrict__ dst = a.out + (size_t)z * H * W;

    const int rh = (WH > 0 ? WH : a.win_h) / 2, rw = (WW > 0 ? WW : a.win_w) / 2;
    const int tw = kBX + 2 * rw, th = kBY + 2 * rh;
    const int x0 = bx * kBX - rw, y0 = by * kBY - rh;
    for (int i = threadIdx.x; i < tw * th; i += 256) {
        const int ty = i / tw, tx = i - ty * tw;
        const int y = clampi(y0 + ty, 0, H - 1), x = clampi(x0 + tx, 0, W - 1);
        tile[ty * tw + tx] = ld(img + (size_t)y * a.pitch + x);
    }
    __syncthreads();

    const int lx = threadIdx.x % kBX, ly = threadIdx.x / kBX;
    const int u = bx * kBX + lx, v = by * kBY + ly;
    if (u >= W || v >= H) return;
    const float* win = tile + ly * tw + lx;
    uint64_t bits;
    if constexpr (WH > 0) bits = census_fixed<WH, WW>(win);
    else if constexpr (WH < 0) bits = census_listed(win, a, tw, rh * tw + rw);
    else bits = census_any(win, a.win_h, a.win_w, tw);
    dst[(size_t)v * W + u] = bits;
}

// WH = WW = 0: any dense window (sizes from the arguments); -1: a listed
// (sparse) neighbour set inside the win_h x win_w window
template <class Src, typename T, int WH, int WW>
__global__ __launch_bounds__(256) void census_kernel(Src src) {
    __shared__ float tile[(kBY + 2 * kMaxCensusRadius) * (kBX + 2 * kMaxCensusRadius)];
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const CensusArgs& a = member_ref(src, vb, b);   // off[] is indexed by image
        __syncthreads();                          // the tile of the previous block is read
        census_block<T, WH, WW>(a, b, tile);
    }
}

uint32_t census_blocks(const CensusArgs& a) {
    return (uint32_t)a.bx * a.by * a.n;
}

CensusArgs census_args(const void* base, int H, int W, int pitch, const lf_census_window& w,
                       uint64_t* out) {
    CensusArgs a{};
    a.base = base;
    a.H = H;
    a.W = W;
    a.pitch = pitch;
    a.win_h = w.win_h;
    a.win_w = w.win_w;
    // offsets validated by the caller: |dy| <= win_h/2, |dx| <= win_w/2
    const int rh = w.win_h / 2, rw = w.win_w / 2;
    a.ntap = w.n_offsets;
    for (int n = 0; n < w.n_offsets; ++n)
        a.tap[n] = (uint8_t)((rh + w.dy[n]) | (rw + w.dx[n]) << 4);
    a.bx = (W + kBX - 1) / kBX;
    a.by = (H + kBY - 1) / kBY;
    a.out = out;
    return a;
}

template <typename T, int WH, int WW>
hipError_t census_variant(Runner& r, int stage, const std::vector<CensusArgs>& args,
                          const std::vector<uint32_t>& blocks) {
    return launch(r, stage, census_kernel<Single<CensusArgs>, T, WH, WW>,
                  census_kernel<Group<CensusArgs>, T, WH, WW>, args, blocks, 256);
}

// One launch per input type and window size (the 5x5 and 7x9 windows of the
// workloads compiled for their size, any other dense window through the general
// loop, listed neighbour sets through the tap loop).
template <typename T>
hipError_t census_windows(Runner& r, int stage, const std::vector<CensusArgs>& args) {
    std::vector<CensusArgs> by[4];
    std::vector<uint32_t> blocks[4];
    for (const CensusArgs& a : args) {
        const int w = a.ntap > 0                       ? 3
                      : a.win_h == 5 && a.win_w == 5 ? 0
                      : a.win_h == 7 && a.win_w == 9 ? 1
                                                     : 2;
        by[w].push_back(a);
        blocks[w].push_back(census_blocks(a));
    }
    hipError_t e = hipSuccess;
    if (!by[0].empty() && (e = census_variant<T, 5, 5>(r, stage, by[0], blocks[0])) != hipSuccess)
        return e;
    if (!by[1].empty() && (e = census_variant<T, 7, 9>(r, stage, by[1], blocks[1])) != hipSuccess)
        return e;
    if (!by[2].empty() && (e = census_variant<T, 0, 0>(r, stage, by[2], blocks[2])) != hipSuccess)
        return e;
    if (!by[3].empty()) e = census_variant<T, -1, -1>(r, stage, by[3], blocks[3]);
    return e;
}

hipError_t launch_census(Runner& r, int stage, int dtype, const std::vector<CensusArgs>& args) {
    return dtype == LF_U8 ? census_windows<uint8_t>(r, stage, args)
                          : census_windows<float>(r, stage, args);
}

}  // namespace

hipError_t census_image(Runner& r, const void* img, int dtype, int H, int W, int pitch,
                        const lf_census_window& win, uint64_t* out) {
    CensusArgs a = census_args(img, H, W, pitch, win, out);
    a.n = 1;
    a.off[0] = 0;
    return launch_census(r, kStCensus, dtype, {a});
}

hipError_t stage_census(Runner& r, const Jobs& jobs, bool all_views) {
    std::vector<CensusArgs> by_type[2];
    for (const Job* j : jobs) {
        // a view is C planes of H x pitch; image z of the output is plane z % C of
        // view z / C (reference first, then the cross views; or all views)
        const int C = j->C;
        const int64_t ps = (int64_t)j->H * j->pitch;            // plane stride
        CensusArgs a = census_args(j->views, j->H, j->W, j->pitch, j->prm.census,
                                   all_views ? j->census_all : j->census);
        if (all_views) {
            a.n = j->S * j->T * C;
            a.stride = ps;
            for (int z = 0; z < a.n && z < kMaxBatchImages; ++z) a.off[z] = z * ps;
        } else {
            const int sh = (j->S - 1) / 2, th = (j->T - 1) / 2;
            a.n = (1 + j->nv) * C;                               // <= 5 * 3 images
            for (int c = 0; c < C; ++c) {
                a.off[c] = (((int64_t)th * j->S + sh) * C + c) * ps;
                for (int i = 0; i < j->nv; ++i)
                    a.off[(1 + i) * C + c] =
                        (((int64_t)j->st[2 * i + 1] * j->S + j->st[2 * i]) * C + c) * ps;
            }
        }
        by_type[j->dtype == LF_U8 ? 0 : 1].push_back(a);
    }
    const int stage = all_views ? kStCostInputs : kStCensus;
    for (int t = 0; t < 2; ++t) {
        if (by_type[t].empty()) continue;
        hipError_t e = launch_census(r, stage, t == 0 ? LF_U8 : LF_F32, by_type[t]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lf
