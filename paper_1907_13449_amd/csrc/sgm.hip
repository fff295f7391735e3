// Semi-global matching, Eq. (8)-(10), on gfx950.
//
// Schedule: one wavefront per path line; lane l holds the hypotheses
// k = K*l .. K*l+K-1 (K = ceil(N/64)), so the path state of one pixel lives in
// the registers of one wave.  Per step along the line:
//   - the matching cost of the K hypotheses (initial stage: Hamming distance of
//     the reference Census string and the view's string at the rounded shift,
//     computed on the fly with popcount; final stage: read from the CSR volume);
//   - the neighbours k-1 / k+1 of the previous pixel's state come from the own
//     registers or, at the lane boundary, from lane l-1 / l+1 by a DPP wave
//     shift (wave_shr:1 / wave_shl:1);
//   - m = min_k L_r(p-r, k) is a DPP reduction (quad perms, half/row mirror,
//     row broadcasts) followed by a readlane, so it is wave-uniform in an SGPR;
//   - the path cost is added into the aggregated volume C_s.
// Path costs use the normalised recurrence (L - m), which stays in [0, C + P2];
// hypotheses outside a pixel's range hold +inf (kInf) so they never win a min
// and the min over the range of p-r is the min over the whole wave.
// The directions run as separate launches (each line of one direction touches
// distinct pixels, so the read-modify-write of C_s needs no atomics); the last
// launch of the initial stage fuses the WTA of Eq. (10).
#include "lf_internal.h"

#include <climits>

namespace lf {
namespace {

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// Minimum over the 64 lanes, returned wave-uniform.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = min(v, dpp<0xB1>(v, v));        // quad_perm [1,0,3,2]
    v = min(v, dpp<0x4E>(v, v));        // quad_perm [2,3,0,1]
    v = min(v, dpp<0x141>(v, v));       // row_half_mirror
    v = min(v, dpp<0x140>(v, v));       // row_mirror: every lane holds its row's min
    v = min(v, dpp<0x142, 0xA>(v, v));  // row_bcast:15 into rows 1, 3
    v = min(v, dpp<0x143, 0xC>(v, v));  // row_bcast:31 into rows 2, 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Start pixel and length of path line `line` of direction (du, dv).
__device__ __forceinline__ void line_start(int H, int W, int du, int dv, int line, int& u0,
                                           int& v0, int& len) {
    if (dv == 0) {                       // horizontal: one line per row
        u0 = du > 0 ? 0 : W - 1;
        v0 = line;
        len = W;
    } else if (du == 0) {                // vertical: one line per column
        u0 = line;
        v0 = dv > 0 ? 0 : H - 1;
        len = H;
    } else {                             // diagonal: entries on a row, then on a column
        if (line < W) {
            u0 = line;
            v0 = dv > 0 ? 0 : H - 1;
        } else {
            const int j = line - W + 1;
            u0 = du > 0 ? 0 : W - 1;
            v0 = dv > 0 ? j : H - 1 - j;
        }
        const int lu = du > 0 ? W - u0 : u0 + 1;
        const int lv = dv > 0 ? H - v0 : v0 + 1;
        len = min(lu, lv);
    }
}

__host__ __device__ inline int num_lines(int H, int W, int du, int dv) {
    return dv == 0 ? H : (du == 0 ? W : W + H - 1);
}

enum { kFirst = 0, kMid = 1, kLastWta = 2 };
constexpr int kWavesPerBlock = 4;

// One step of the normalised recurrence for K consecutive hypotheses.
template <int K>
__device__ __forceinline__ void sgm_step(const uint32_t (&Lp)[K], uint32_t m, uint32_t P1,
                                         uint32_t P2, const uint32_t (&C)[K],
                                         const bool (&valid)[K], uint32_t (&L)[K]) {
    const uint32_t left = dpp<0x138>(kInf, Lp[K - 1]);   // wave_shr:1 -> from lane l-1
    const uint32_t right = dpp<0x130>(kInf, Lp[0]);      // wave_shl:1 -> from lane l+1
    const uint32_t mP2 = m + P2;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint32_t lm = j == 0 ? left : Lp[j - 1];
        const uint32_t lp = j == K - 1 ? right : Lp[j + 1];
        const uint32_t t = min(min(Lp[j], mP2), min(lm, lp) + P1);
        L[j] = valid[j] ? C[j] + (t - m) : kInf;
    }
}

// Initial stage: Census cost on the fly, every hypothesis, views on blockIdx.y.
template <int K, int PHASE>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sgm_dense_kernel(
    SgmDense a, const float* __restrict__ hyp, int H, int W, int N, uint32_t P1, uint32_t P2,
    int du, int dv) {
    const int lane = threadIdx.x & 63;
    const int line = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (line >= num_lines(H, W, du, dv)) return;       // wave-uniform exit
    const int z = blockIdx.y;
    int u0, v0, len;
    line_start(H, W, du, dv, line, u0, v0, len);
    const size_t HW = (size_t)H * W;
    const uint64_t* __restrict__ cref = a.cref;
    const uint64_t* __restrict__ cv = a.cview + (size_t)z * HW;
    uint16_t* __restrict__ csum = a.csum + (size_t)z * HW * N;

    int ku[K], kv[K];
    bool valid[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int k = lane * K + j;
        valid[j] = k < N;
        const float d = hyp[min(k, N - 1)];
        ku[j] = (int)rintf((float)a.cs[z] * d);
        kv[j] = (int)rintf((float)a.ct[z] * d);
    }
    uint32_t Lp[K], m = 0;
    for (int step = 0; step < len; ++step) {
        const int u = u0 + step * du, v = v0 + step * dv;
        const size_t p = (size_t)v * W + u;
        const uint64_t cr = cref[p];
        uint32_t C[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int x = clampi(u + ku[j], 0, W - 1), y = clampi(v + kv[j], 0, H - 1);
            C[j] = (uint32_t)__popcll(cr ^ cv[(size_t)y * W + x]);
        }
        uint32_t L[K];
        if (step == 0) {
#pragma unroll
            for (int j = 0; j < K; ++j) L[j] = valid[j] ? C[j] : kInf;
        } else {
            sgm_step<K>(Lp, m, P1, P2, C, valid, L);
        }
        uint32_t mn = L[0];
#pragma unroll
        for (int j = 1; j < K; ++j) mn = min(mn, L[j]);
        m = wave_min(mn);

        uint16_t* row = csum + p * N + lane * K;
        if (PHASE == kFirst) {
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (valid[j]) row[j] = (uint16_t)L[j];
        } else if (PHASE == kMid) {
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (valid[j]) row[j] = (uint16_t)(row[j] + L[j]);
        } else {
            uint32_t key = UINT_MAX;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (valid[j]) key = min(key, ((row[j] + L[j]) << 8) | (uint32_t)(lane * K + j));
            key = wave_min(key);
            if (lane == 0) a.dmap[(size_t)z * HW + p] = (int16_t)(key & 0xFF);
        }
#pragma unroll
        for (int j = 0; j < K; ++j) Lp[j] = L[j];
    }
}

// Final stage: CSR volume over per-pixel ranges [lo, hi].
template <int K, int PHASE, typename SumT>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sgm_bounded_kernel(
    SgmBounded a, int H, int W, uint32_t P1, uint32_t P2, int du, int dv) {
    const int lane = threadIdx.x & 63;
    const int line = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (line >= num_lines(H, W, du, dv)) return;
    int u0, v0, len;
    line_start(H, W, du, dv, line, u0, v0, len);
    const uint16_t* __restrict__ cost = a.cost;
    SumT* __restrict__ csum = reinterpret_cast<SumT*>(a.csum);

    uint32_t Lp[K], m = 0;
    for (int step = 0; step < len; ++step) {
        const int u = u0 + step * du, v = v0 + step * dv;
        const size_t p = (size_t)v * W + u;
        const int lo = a.lo[p], hi = a.hi[p];
        const int64_t base = a.off[p] - lo;
        uint32_t C[K];
        bool valid[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int k = lane * K + j;
            valid[j] = k >= lo && k <= hi;
            C[j] = valid[j] ? (uint32_t)cost[base + k] : 0u;
        }
        uint32_t L[K];
        if (step == 0) {
#pragma unroll
            for (int j = 0; j < K; ++j) L[j] = valid[j] ? C[j] : kInf;
        } else {
            sgm_step<K>(Lp, m, P1, P2, C, valid, L);
        }
        uint32_t mn = L[0];
#pragma unroll
        for (int j = 1; j < K; ++j) mn = min(mn, L[j]);
        m = wave_min(mn);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!valid[j]) continue;
            SumT* c = csum + base + lane * K + j;
            *c = PHASE == kFirst ? (SumT)L[j] : (SumT)(*c + L[j]);
        }
#pragma unroll
        for (int j = 0; j < K; ++j) Lp[j] = L[j];
    }
}

const int kDirs[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};

template <int K>
hipError_t dense_passes(const SgmDense& a, const float* hyp, int H, int W, int N, int P1,
                        int P2, int npaths, hipStream_t st) {
    for (int r = 0; r < npaths; ++r) {
        const int du = kDirs[r][0], dv = kDirs[r][1];
        dim3 grid((num_lines(H, W, du, dv) + kWavesPerBlock - 1) / kWavesPerBlock, a.nv);
        dim3 block(64 * kWavesPerBlock);
        if (r == 0)
            hipLaunchKernelGGL((sgm_dense_kernel<K, kFirst>), grid, block, 0, st, a, hyp, H, W,
                               N, (uint32_t)P1, (uint32_t)P2, du, dv);
        else if (r + 1 < npaths)
            hipLaunchKernelGGL((sgm_dense_kernel<K, kMid>), grid, block, 0, st, a, hyp, H, W, N,
                               (uint32_t)P1, (uint32_t)P2, du, dv);
        else
            hipLaunchKernelGGL((sgm_dense_kernel<K, kLastWta>), grid, block, 0, st, a, hyp, H,
                               W, N, (uint32_t)P1, (uint32_t)P2, du, dv);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int K, typename SumT>
hipError_t bounded_passes(const SgmBounded& a, int H, int W, int P1, int P2, int npaths,
                          hipStream_t st) {
    for (int r = 0; r < npaths; ++r) {
        const int du = kDirs[r][0], dv = kDirs[r][1];
        dim3 grid((num_lines(H, W, du, dv) + kWavesPerBlock - 1) / kWavesPerBlock);
        dim3 block(64 * kWavesPerBlock);
        if (r == 0)
            hipLaunchKernelGGL((sgm_bounded_kernel<K, kFirst, SumT>), grid, block, 0, st, a, H,
                               W, (uint32_t)P1, (uint32_t)P2, du, dv);
        else
            hipLaunchKernelGGL((sgm_bounded_kernel<K, kMid, SumT>), grid, block, 0, st, a, H, W,
                               (uint32_t)P1, (uint32_t)P2, du, dv);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_sgm_dense(const SgmDense& a, const float* hyp, int H, int W, int N, int P1,
                            int P2, int npaths, hipStream_t st) {
    switch ((N + 63) / 64) {
        case 1: return dense_passes<1>(a, hyp, H, W, N, P1, P2, npaths, st);
        case 2: return dense_passes<2>(a, hyp, H, W, N, P1, P2, npaths, st);
        case 3: return dense_passes<3>(a, hyp, H, W, N, P1, P2, npaths, st);
        default: return dense_passes<4>(a, hyp, H, W, N, P1, P2, npaths, st);
    }
}

hipError_t launch_sgm_bounded(const SgmBounded& a, int H, int W, int N, int P1, int P2,
                              int npaths, hipStream_t st) {
    const int K = (N + 63) / 64;
    if (a.sum_bits == 16) {
        switch (K) {
            case 1: return bounded_passes<1, uint16_t>(a, H, W, P1, P2, npaths, st);
            case 2: return bounded_passes<2, uint16_t>(a, H, W, P1, P2, npaths, st);
            case 3: return bounded_passes<3, uint16_t>(a, H, W, P1, P2, npaths, st);
            default: return bounded_passes<4, uint16_t>(a, H, W, P1, P2, npaths, st);
        }
    }
    switch (K) {
        case 1: return bounded_passes<1, uint32_t>(a, H, W, P1, P2, npaths, st);
        case 2: return bounded_passes<2, uint32_t>(a, H, W, P1, P2, npaths, st);
        case 3: return bounded_passes<3, uint32_t>(a, H, W, P1, P2, npaths, st);
        default: return bounded_passes<4, uint32_t>(a, H, W, P1, P2, npaths, st);
    }
}

}  // namespace lf
