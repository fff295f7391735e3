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

template <typename T>
__global__ __launch_bounds__(256) void census_kernel(CensusBatch b, int H, int W, int pitch,
                                                     int win_h, int win_w,
                                                     uint64_t* __restrict__ out) {
    __shared__ float tile[(kBY + 2 * kMaxCensusRadius) * (kBX + 2 * kMaxCensusRadius)];
    const int z = blockIdx.z;
    const int64_t off = b.n > kMaxBatchImages ? (int64_t)z * b.stride : b.off[z];
    const T* __restrict__ img = reinterpret_cast<const T*>(b.base) + off;
    uint64_t* __restrict__ dst = out + (size_t)z * H * W;

    const int rh = win_h / 2, rw = win_w / 2;
    const int tw = kBX + 2 * rw, th = kBY + 2 * rh;
    const int x0 = blockIdx.x * kBX - rw, y0 = blockIdx.y * kBY - rh;
    for (int i = threadIdx.x; i < tw * th; i += 256) {
        const int ty = i / tw, tx = i - ty * tw;
        const int y = clampi(y0 + ty, 0, H - 1), x = clampi(x0 + tx, 0, W - 1);
        tile[ty * tw + tx] = ld(img + (size_t)y * pitch + x);
    }
    __syncthreads();

    const int lx = threadIdx.x % kBX, ly = threadIdx.x / kBX;
    const int u = blockIdx.x * kBX + lx, v = blockIdx.y * kBY + ly;
    if (u >= W || v >= H) return;
    const float c = tile[(ly + rh) * tw + lx + rw];
    uint64_t bits = 0;
    int n = 0;
    for (int i = 0; i < win_h; ++i) {
        const float* row = tile + (ly + i) * tw + lx;
        for (int j = 0; j < win_w; ++j) {
            if (i == rh && j == rw) continue;
            bits |= (uint64_t)(c > row[j]) << n;
            ++n;
        }
    }
    dst[(size_t)v * W + u] = bits;
}

}  // namespace

hipError_t launch_census(const CensusBatch& b, int dtype, int H, int W, int pitch, int win_h,
                         int win_w, uint64_t* out, hipStream_t st) {
    dim3 grid((W + kBX - 1) / kBX, (H + kBY - 1) / kBY, b.n);
    if (dtype == LF_U8)
        hipLaunchKernelGGL(census_kernel<uint8_t>, grid, dim3(256), 0, st, b, H, W, pitch,
                           win_h, win_w, out);
    else
        hipLaunchKernelGGL(census_kernel<float>, grid, dim3(256), 0, st, b, H, W, pitch, win_h,
                           win_w, out);
    return hipGetLastError();
}

}  // namespace lf
