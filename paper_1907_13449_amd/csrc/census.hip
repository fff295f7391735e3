// Census transform, Sec. 3.2 Eq. (2)-(3), from LDS-staged tiles.
//
// A 256-thread workgroup owns a 32 x 8 pixel tile.  It stages the tile plus the
// window halo (clamp-to-edge) into LDS once, as float, with coalesced row loads,
// then each thread compares its centre with the win_h*win_w - 1 neighbours in
// row-major order (centre skipped), bit n = [centre > neighbour n].
#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kBX = 32, kBY = 8;

// Up to kMaxBatchImages images of one size; image z starts at base + off[z]
// elements, or at base + z * stride when n > kMaxBatchImages.
struct CensusArgs {
    const void* base;
    int64_t off[kMaxBatchImages];
    int64_t stride;
    int n;
    int H, W, pitch, win_h, win_w;
    int bx, by;               // tiles along x and y
    uint64_t* out;            // [n][H*W]
};

template <typename T>
__device__ __forceinline__ void census_block(const CensusArgs& a, uint32_t b, float* tile) {
    const int per = a.bx * a.by;
    const int z = (int)b / per;
    const int rem = (int)b - z * per;
    const int by = rem / a.bx, bx = rem - by * a.bx;
    const int H = a.H, W = a.W;
    const int64_t off = a.n > kMaxBatchImages ? (int64_t)z * a.stride : a.off[z];
    const T* __restrict__ img = reinterpret_cast<const T*>(a.base) + off;
    uint64_t* __restrict__ dst = a.out + (size_t)z * H * W;

    const int rh = a.win_h / 2, rw = a.win_w / 2;
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
    const float c = tile[(ly + rh) * tw + lx + rw];
    uint64_t bits = 0;
    int n = 0;
    for (int i = 0; i < a.win_h; ++i) {
        const float* row = tile + (ly + i) * tw + lx;
        for (int j = 0; j < a.win_w; ++j) {
            if (i == rh && j == rw) continue;
            bits |= (uint64_t)(c > row[j]) << n;
            ++n;
        }
    }
    dst[(size_t)v * W + u] = bits;
}

template <class Src, typename T>
__global__ __launch_bounds__(256) void census_kernel(Src src) {
    __shared__ float tile[(kBY + 2 * kMaxCensusRadius) * (kBX + 2 * kMaxCensusRadius)];
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const CensusArgs& a = member(src, vb, b);
        __syncthreads();                          // the tile of the previous block is read
        census_block<T>(a, b, tile);
    }
}

uint32_t census_blocks(const CensusArgs& a) {
    return (uint32_t)a.bx * a.by * a.n;
}

CensusArgs census_args(const void* base, int H, int W, int pitch, int win_h, int win_w,
                       uint64_t* out) {
    CensusArgs a{};
    a.base = base;
    a.H = H;
    a.W = W;
    a.pitch = pitch;
    a.win_h = win_h;
    a.win_w = win_w;
    a.bx = (W + kBX - 1) / kBX;
    a.by = (H + kBY - 1) / kBY;
    a.out = out;
    return a;
}

hipError_t launch_census(Runner& r, int stage, int dtype, const std::vector<CensusArgs>& args) {
    std::vector<uint32_t> blocks;
    for (const CensusArgs& a : args) blocks.push_back(census_blocks(a));
    if (dtype == LF_U8)
        return launch(r, stage, census_kernel<Single<CensusArgs>, uint8_t>,
                      census_kernel<Group<CensusArgs>, uint8_t>, args, blocks, 256);
    return launch(r, stage, census_kernel<Single<CensusArgs>, float>,
                  census_kernel<Group<CensusArgs>, float>, args, blocks, 256);
}

}  // namespace

hipError_t census_image(Runner& r, const void* img, int dtype, int H, int W, int pitch,
                        int win_h, int win_w, uint64_t* out) {
    CensusArgs a = census_args(img, H, W, pitch, win_h, win_w, out);
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
        CensusArgs a = census_args(j->views, j->H, j->W, j->pitch, j->prm.census.win_h,
                                   j->prm.census.win_w, all_views ? j->census_all : j->census);
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
    const int stage = all_views ? kStCost : kStCensus;
    for (int t = 0; t < 2; ++t) {
        if (by_type[t].empty()) continue;
        hipError_t e = launch_census(r, stage, t == 0 ? LF_U8 : LF_F32, by_type[t]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lf
