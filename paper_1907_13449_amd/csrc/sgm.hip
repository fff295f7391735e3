// Semi-global matching, Eq. (8)-(10), on gfx950.
//
// Schedule.  All path directions of all views run in ONE launch: a wavefront
// owns one path line of one direction of one view, and writes that direction's
// path costs L_r to a buffer of its own (no read-modify-write, no atomics); a
// second kernel sums the directions, Eq. (9), and for the initial stage takes
// the WTA of Eq. (10) in the same pass.  With 8 directions x |V| views the launch
// has enough independent waves to keep every SIMD busy while each wave walks its
// line step by step.
//
// Inside a wave, lane l holds hypotheses k = K*l .. K*l+K-1 (K = ceil(N/64)), so
// the state of one pixel lives in the registers of one wave.  Per step:
//   - the matching cost of the K hypotheses, read from a cost volume whose row of
//     the pixel is contiguous (initial stage: the 8-bit Census cost volume, built
//     once by a popcount kernel; final stage: the CSR volume), with the loads of
//     the next kDepth steps in flight;
//   - the neighbours k-1 / k+1 of the previous pixel come from the lane's own
//     registers or, at the lane boundary, from lane l-1 / l+1 by a DPP wave
//     shift (wave_shr:1 / wave_shl:1);
//   - m = min_k L_r(p-r, k) is a DPP reduction (quad perms, half/row mirror, row
//     broadcasts) and a readlane, so it is wave-uniform in an SGPR.
// Path costs use the normalised recurrence (subtract m), which keeps them in
// [0, C + P2]: 8 bits suffice for the Census stage when bits + P2 <= 255.
// Hypotheses outside a pixel's range hold +inf (kInf) so they never win a min.
#include "lf_internal.h"

#include <algorithm>
#include <climits>

namespace lf {
namespace {

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// Minimum over the 64 lanes, returned wave-uniform.
// The DPP source operand "old" is UINT_MAX, the identity of umin, so that each
// move fuses into the v_min_u32 that consumes it (one v_min_u32_dpp per stage).
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = min(v, dpp<0xB1>(UINT_MAX, v));        // quad_perm [1,0,3,2]
    v = min(v, dpp<0x4E>(UINT_MAX, v));        // quad_perm [2,3,0,1]
    v = min(v, dpp<0x141>(UINT_MAX, v));       // row_half_mirror
    v = min(v, dpp<0x140>(UINT_MAX, v));       // row_mirror: every lane holds its row's min
    v = min(v, dpp<0x142, 0xA>(UINT_MAX, v));  // row_bcast:15 into rows 1, 3
    v = min(v, dpp<0x143, 0xC>(UINT_MAX, v));  // row_bcast:31 into rows 2, 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

const int kDirs[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};

__host__ __device__ inline int num_lines(int H, int W, int du, int dv) {
    return dv == 0 ? H : (du == 0 ? W : W + H - 1);
}

// Lines of every direction, numbered consecutively: direction r owns global
// lines [base[r], base[r+1]).
struct Lines {
    int base[9];
    int du[8], dv[8];
    int npaths;
};

Lines make_lines(int H, int W, int npaths) {
    Lines L{};
    L.npaths = npaths;
    L.base[0] = 0;
    for (int r = 0; r < npaths; ++r) {
        L.du[r] = kDirs[r][0];
        L.dv[r] = kDirs[r][1];
        L.base[r + 1] = L.base[r] + num_lines(H, W, L.du[r], L.dv[r]);
    }
    return L;
}

struct LineInfo {
    int r, u0, v0, du, dv, len;
};

__device__ __forceinline__ LineInfo locate(const Lines& L, int H, int W, int g) {
    LineInfo li;
    int r = 0;
#pragma unroll
    for (int i = 1; i < 8; ++i) r += (i < L.npaths && g >= L.base[i]) ? 1 : 0;
    const int line = g - L.base[r];
    const int du = L.du[r], dv = L.dv[r];
    li.r = r;
    li.du = du;
    li.dv = dv;
    if (dv == 0) {                       // horizontal: one line per row
        li.u0 = du > 0 ? 0 : W - 1;
        li.v0 = line;
        li.len = W;
    } else if (du == 0) {                // vertical: one line per column
        li.u0 = line;
        li.v0 = dv > 0 ? 0 : H - 1;
        li.len = H;
    } else {                             // diagonal: entries on a row, then on a column
        if (line < W) {
            li.u0 = line;
            li.v0 = dv > 0 ? 0 : H - 1;
        } else {
            const int j = line - W + 1;
            li.u0 = du > 0 ? 0 : W - 1;
            li.v0 = dv > 0 ? j : H - 1 - j;
        }
        const int lu = du > 0 ? W - li.u0 : li.u0 + 1;
        const int lv = dv > 0 ? H - li.v0 : li.v0 + 1;
        li.len = min(lu, lv);
    }
    return li;
}

constexpr int kWavesPerBlock = 4;
constexpr int kDepth = 8;          // steps of input prefetched ahead of the recurrence

// Copies a wave-uniform value into a VGPR that the compiler treats as divergent.
// Loads addressed through it stay vector-memory loads, which complete in order,
// so a wave can keep several steps of them in flight and wait for the oldest
// only (scalar loads can only be awaited all at once).
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x) {
    asm volatile("" : "=v"(x) : "0"(x));
    return x;
}

// One step of the normalised recurrence for K consecutive hypotheses.  Lanes
// whose hypotheses do not exist carry costs >= kInf and so path costs >= kInf,
// which never win a min; the neighbour shift brings UINT_MAX (the identity of
// umin) in at the wave edges.
template <int K>
__device__ __forceinline__ void sgm_step(const uint32_t (&Lp)[K], uint32_t m, uint32_t P1,
                                         uint32_t P2, const uint32_t (&C)[K], uint32_t (&L)[K]) {
    const uint32_t left = dpp<0x138>(UINT_MAX, Lp[K - 1]);   // wave_shr:1 -> from lane l-1
    const uint32_t right = dpp<0x130>(UINT_MAX, Lp[0]);      // wave_shl:1 -> from lane l+1
    const uint32_t mP2 = m + P2;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint32_t lm = j == 0 ? left : Lp[j - 1];
        const uint32_t lp = j == K - 1 ? right : Lp[j + 1];
        const uint32_t t = min(min(Lp[j], mP2), min(lm, lp) + P1);
        L[j] = C[j] + (t - m);
    }
}

template <int K>
__device__ __forceinline__ uint32_t lane_min(const uint32_t (&L)[K]) {
    uint32_t mn = L[0];
#pragma unroll
    for (int j = 1; j < K; ++j) mn = min(mn, L[j]);
    return mn;
}

// ---------------------------------------------------------------------------
// Initial stage, Eq. (7): the Census cost volume C[z][p][NP] (8-bit, NP = N
// rounded up to 4) of every cross view, computed once and read by all path
// directions.  A workgroup builds the tile of 64 consecutive pixels x NP
// hypotheses in LDS with lanes over pixels -- for a fixed hypothesis the 64
// gathered Census strings are consecutive in memory for both shift axes -- and
// then writes the tile, which is contiguous in C, with 32-bit stores.
constexpr int kTilePix = 64;

__global__ __launch_bounds__(256) void census_cost_volume_kernel(SgmDense a,
                                                                 const float* __restrict__ hyp,
                                                                 int H, int W, int N, int NP,
                                                                 uint8_t* __restrict__ cvol) {
    __shared__ uint32_t tile[kTilePix * LF_MAX_HYPOTHESES / 4];
    __shared__ int s_sh[LF_MAX_HYPOTHESES];
    const int z = blockIdx.y;
    const uint32_t HW = (uint32_t)H * W;
    const uint32_t p0 = blockIdx.x * kTilePix;
    const int npix = (int)min((uint32_t)kTilePix, HW - p0);
    const bool along_u = a.ct[z] == 0;
    const int cs = along_u ? a.cs[z] : a.ct[z];
    for (int k = threadIdx.x; k < NP; k += 256)
        s_sh[k] = (int)rintf((float)cs * hyp[min(k, N - 1)]);
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t p = p0 + (uint32_t)min(lane, npix - 1);
    const int v = (int)(p / W), u = (int)(p - (uint32_t)v * W);
    const uint64_t r = a.cref[p];
    const uint64_t* __restrict__ cv = a.cview + (size_t)z * HW;
    uint8_t* t8 = (uint8_t*)tile;
    for (int k = wave; k < NP; k += 4) {          // k is wave-uniform
        const int sh = s_sh[k];
        const uint32_t q = along_u ? (uint32_t)(v * W + clampi(u + sh, 0, W - 1))
                                   : (uint32_t)(clampi(v + sh, 0, H - 1) * W + u);
        t8[lane * NP + k] = k < N ? (uint8_t)__popcll(r ^ cv[q]) : (uint8_t)0;
    }
    __syncthreads();
    // the tile is npix * NP contiguous bytes of C (NP is a multiple of 4)
    uint32_t* dst = (uint32_t*)(cvol + ((size_t)z * HW + p0) * NP);
    const int words = npix * NP / 4;
    for (int i = threadIdx.x; i < words; i += 256) dst[i] = tile[i];
}

// SGM over the Census cost volume, every direction of every view in one launch;
// blockIdx.y = view.  Output: Lbuf[r][z][p][NP], storage type LT.
template <int K, typename LT>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sgm_dense_paths_kernel(
    const uint8_t* __restrict__ cvol, int nv, Lines lines, int H, int W, int N, int NP,
    uint32_t P1, uint32_t P2, LT* __restrict__ Lbuf) {
    const int lane = threadIdx.x & 63;
    const int g = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    if (g >= lines.base[lines.npaths]) return;         // wave-uniform exit
    const int z = blockIdx.y;
    const LineInfo li = locate(lines, H, W, g);
    const uint32_t HW = (uint32_t)H * W;
    const uint8_t* __restrict__ cz = cvol + (size_t)z * HW * NP;
    LT* __restrict__ out = Lbuf + ((size_t)li.r * nv + z) * HW * NP;

    // the lane's K bytes of a pixel row; lanes past N read in-row bytes and add kInf
    const uint32_t lofs = (uint32_t)min(lane * K, NP - K);
    uint32_t cinit[K];
#pragma unroll
    for (int j = 0; j < K; ++j) cinit[j] = lane * K + j < N ? 0u : kInf;
    const int last = li.len - 1;
    auto load = [&](int step) -> uint32_t {
        step = min(step, last);
        const uint32_t p = (uint32_t)((li.v0 + step * li.dv) * W + li.u0 + step * li.du);
        const uint32_t o = p * (uint32_t)NP + lofs;      // 32-bit offset off a scalar base
        if constexpr (K == 1) return cz[o];
        else if constexpr (K == 2) return *(const uint16_t*)(cz + o);
        else if constexpr (K == 4) return *(const uint32_t*)(cz + o);
        else return (uint32_t)cz[o] | ((uint32_t)cz[o + 1] << 8) | ((uint32_t)cz[o + 2] << 16);
    };
    uint32_t cb[kDepth];
#pragma unroll
    for (int i = 0; i < kDepth; ++i) cb[i] = load(i);

    uint32_t Lp[K], m = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) Lp[j] = kInf;
    for (int base = 0; base < li.len; base += kDepth) {
#pragma unroll
        for (int i = 0; i < kDepth; ++i) {
            const int step = base + i;           // steps past the line end are computed
            uint32_t C[K];                       // and not stored
#pragma unroll
            for (int j = 0; j < K; ++j) C[j] = ((cb[i] >> (8 * j)) & 0xFFu) + cinit[j];
            cb[i] = load(step + kDepth);         // refill the slot just consumed
            uint32_t L[K];
            if (step == 0) {
#pragma unroll
                for (int j = 0; j < K; ++j) L[j] = C[j];
            } else {
                sgm_step<K>(Lp, m, P1, P2, C, L);
            }
            m = wave_min(lane_min(L));

            const uint32_t p = (uint32_t)((li.v0 + step * li.dv) * W + li.u0 + step * li.du);
            const uint32_t e0 = p * (uint32_t)NP + (uint32_t)(lane * K);   // element offset
            if (step < li.len) {
                if constexpr (K == 2) {
                    if (lane * 2 < N) {          // a pair: one 16- or 32-bit store
                        if constexpr (sizeof(LT) == 1)
                            *(uint16_t*)(out + e0) = (uint16_t)((L[0] & 0xFF) | (L[1] << 8));
                        else
                            *(uint32_t*)(out + e0) = (L[0] & 0xFFFF) | (L[1] << 16);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < K; ++j)
                        if (lane * K + j < N) out[e0 + j] = (LT)L[j];
                }
            }
#pragma unroll
            for (int j = 0; j < K; ++j) Lp[j] = L[j];
        }
    }
}

// Sum over directions + WTA (Eq. 9-10) of the initial stage: one wave per pixel,
// lane l holds hypotheses 2l and 2l+1 (+128 per round); lowest index on ties.
template <typename LT>
__global__ __launch_bounds__(256) void dense_sum_wta_kernel(const LT* __restrict__ Lbuf,
                                                            int npaths, int nv, int64_t HW,
                                                            int N, int NP,
                                                            int16_t* __restrict__ dmap) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const size_t dir_stride = (size_t)nv * HW * NP;
    for (int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); q < nv * HW; q += nwaves) {
        const LT* base = Lbuf + (size_t)q * NP;        // q = z*HW + p
        uint32_t key = UINT_MAX;
        for (int k = 2 * lane; k < N; k += 128) {
            uint32_t t0 = 0, t1 = 0;
#pragma unroll 8
            for (int r = 0; r < npaths; ++r) {
                const LT* e = base + (size_t)r * dir_stride + k;
                if constexpr (sizeof(LT) == 1) {
                    const uint32_t x = *(const uint16_t*)e;
                    t0 += x & 0xFF;
                    t1 += x >> 8;
                } else {
                    const uint32_t x = *(const uint32_t*)e;
                    t0 += x & 0xFFFF;
                    t1 += x >> 16;
                }
            }
            key = min(key, (t0 << 8) | (uint32_t)k);
            if (k + 1 < N) key = min(key, (t1 << 8) | (uint32_t)(k + 1));
        }
        key = wave_min(key);
        if (lane == 0) dmap[q] = (int16_t)(key & 0xFF);
    }
}

// ---------------------------------------------------------------------------
// Final stage: CSR volume over per-pixel ranges [lo, hi].  Output Lbuf[r][cell].
// meta[p] = {off[p] - lo[p] (int64), lo | hi << 16}: one 16-byte load per step.
struct alignas(16) PixMeta {
    int64_t base;
    int32_t lohi;
    int32_t pad;
};

__global__ __launch_bounds__(256) void pix_meta_kernel(const int64_t* __restrict__ off,
                                                       const int16_t* __restrict__ lo,
                                                       const int16_t* __restrict__ hi, int HW,
                                                       PixMeta* __restrict__ meta) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= HW) return;
    PixMeta m;
    m.base = off[p] - lo[p];
    m.lohi = (int32_t)((uint16_t)lo[p] | ((uint32_t)(uint16_t)hi[p] << 16));
    m.pad = 0;
    meta[p] = m;
}

template <int K>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sgm_bounded_paths_kernel(
    SgmBounded a, const PixMeta* __restrict__ meta, Lines lines, int H, int W, uint32_t P1,
    uint32_t P2, size_t dir_stride, uint16_t* __restrict__ Lbuf) {
    constexpr int kMeta = kDepth, kCost = kDepth / 2;   // two-stage prefetch
    const int lane = threadIdx.x & 63;
    const int g = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    if (g >= lines.base[lines.npaths]) return;
    const LineInfo li = locate(lines, H, W, g);
    const uint16_t* __restrict__ cost = a.cost;
    uint16_t* __restrict__ out = Lbuf + (size_t)li.r * dir_stride;

    auto load_meta = [&](int step) {
        const int u = li.u0 + step * li.du, v = li.v0 + step * li.dv;
        return meta[in_vgpr((uint32_t)(v * W + u))];
    };
    // gather of the K costs of a pixel; hypotheses outside [lo, hi] read the
    // pixel's first cell and are replaced by kInf when used
    auto load_cost = [&](const PixMeta& pm, uint32_t (&c)[K]) {
        const int lo = pm.lohi & 0xFFFF, hi = pm.lohi >> 16;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int k = min(max(lane * K + j, lo), hi);
            c[j] = cost[pm.base + k];
        }
    };
    PixMeta mb[kMeta];
    uint32_t cb[kCost][K];
#pragma unroll
    for (int i = 0; i < kMeta; ++i) mb[i] = load_meta(min(i, li.len - 1));
#pragma unroll
    for (int i = 0; i < kCost; ++i) load_cost(mb[i], cb[i]);

    uint32_t Lp[K], m = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) Lp[j] = kInf;
    for (int base = 0; base < li.len; base += kMeta) {
#pragma unroll
        for (int i = 0; i < kMeta; ++i) {
            const int step = base + i;           // steps past the line end are computed
            const PixMeta pm = mb[i];            // and not stored
            const int lo = pm.lohi & 0xFFFF, hi = pm.lohi >> 16;
            uint32_t C[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int k = lane * K + j;
                C[j] = (k >= lo && k <= hi) ? cb[i % kCost][j] : kInf;
            }
            // refill: costs for step + kCost (its meta arrived kMeta - kCost steps
            // ago), then the meta slot for step + kMeta
            load_cost(mb[(i + kCost) % kMeta], cb[i % kCost]);
            mb[i] = load_meta(min(step + kMeta, li.len - 1));
            uint32_t L[K];
            if (step == 0) {
#pragma unroll
                for (int j = 0; j < K; ++j) L[j] = C[j];
            } else {
                sgm_step<K>(Lp, m, P1, P2, C, L);
            }
            m = wave_min(lane_min(L));
            const bool live = step < li.len;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int k = lane * K + j;
                if (live && k >= lo && k <= hi) out[pm.base + k] = (uint16_t)L[j];
            }
#pragma unroll
            for (int j = 0; j < K; ++j) Lp[j] = L[j];
        }
    }
}

// csum[c] = sum_r Lbuf[r][c] over the cells of the CSR volume.
template <typename SumT>
__global__ __launch_bounds__(256) void bounded_sum_kernel(const uint16_t* __restrict__ Lbuf,
                                                          int npaths, size_t dir_stride,
                                                          const int64_t* __restrict__ total,
                                                          SumT* __restrict__ csum) {
    const int64_t n = *total;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * 256) {
        uint32_t s = 0;
        for (int r = 0; r < npaths; ++r) s += Lbuf[(size_t)r * dir_stride + c];
        csum[c] = (SumT)s;
    }
}

template <int K, typename LT>
hipError_t dense_launch(const SgmDense& a, const Lines& lines, int H, int W, int N, int NP, int P1,
                        int P2, const uint8_t* cvol, void* Lbuf, hipStream_t st) {
    dim3 grid((lines.base[lines.npaths] + kWavesPerBlock - 1) / kWavesPerBlock, a.nv);
    hipLaunchKernelGGL((sgm_dense_paths_kernel<K, LT>), grid, dim3(64 * kWavesPerBlock), 0, st,
                       cvol, a.nv, lines, H, W, N, NP, (uint32_t)P1, (uint32_t)P2, (LT*)Lbuf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t HW = (int64_t)H * W;
    const int64_t waves = a.nv * HW;
    const int blocks = (int)std::min<int64_t>((waves + 3) / 4, 8192);
    hipLaunchKernelGGL((dense_sum_wta_kernel<LT>), dim3(blocks), dim3(256), 0, st,
                       (const LT*)Lbuf, lines.npaths, a.nv, HW, N, NP, a.dmap);
    return hipGetLastError();
}

template <typename LT>
hipError_t dense_dispatch(const SgmDense& a, const Lines& lines, int H, int W, int N, int NP,
                          int P1, int P2, const uint8_t* cvol, void* Lbuf, hipStream_t st) {
    switch ((N + 63) / 64) {
        case 1: return dense_launch<1, LT>(a, lines, H, W, N, NP, P1, P2, cvol, Lbuf, st);
        case 2: return dense_launch<2, LT>(a, lines, H, W, N, NP, P1, P2, cvol, Lbuf, st);
        case 3: return dense_launch<3, LT>(a, lines, H, W, N, NP, P1, P2, cvol, Lbuf, st);
        default: return dense_launch<4, LT>(a, lines, H, W, N, NP, P1, P2, cvol, Lbuf, st);
    }
}

template <int K>
hipError_t bounded_launch(const SgmBounded& a, const PixMeta* meta, const Lines& lines, int H,
                          int W, int P1, int P2, size_t dir_stride, uint16_t* Lbuf,
                          hipStream_t st) {
    dim3 grid((lines.base[lines.npaths] + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL((sgm_bounded_paths_kernel<K>), grid, dim3(64 * kWavesPerBlock), 0, st, a,
                       meta, lines, H, W, (uint32_t)P1, (uint32_t)P2, dir_stride, Lbuf);
    return hipGetLastError();
}

}  // namespace

int dense_np(int N) { return (N + 3) / 4 * 4; }

static size_t round256(size_t x) { return (x + 255) / 256 * 256; }

size_t sgm_dense_scratch_bytes(int nv, int H, int W, int N, int npaths, int bits, int P2) {
    const size_t lt = bits + P2 <= 255 ? 1 : 2;
    const size_t cv = round256((size_t)nv * H * W * dense_np(N));
    return cv + (size_t)npaths * nv * H * W * dense_np(N) * lt;
}

size_t sgm_bounded_scratch_bytes(int H, int W, int N, int npaths) {
    const size_t meta = ((size_t)H * W * sizeof(PixMeta) + 255) / 256 * 256;
    return meta + (size_t)npaths * H * W * N * sizeof(uint16_t);
}

hipError_t launch_sgm_dense(const SgmDense& a, const float* hyp, int H, int W, int N, int P1,
                            int P2, int npaths, int bits, void* scratch, hipStream_t st) {
    const Lines lines = make_lines(H, W, npaths);
    const int NP = dense_np(N);
    uint8_t* cvol = (uint8_t*)scratch;
    void* Lbuf = (char*)scratch + round256((size_t)a.nv * H * W * NP);
    const uint32_t tiles = ((uint32_t)H * W + kTilePix - 1) / kTilePix;
    hipLaunchKernelGGL(census_cost_volume_kernel, dim3(tiles, a.nv), dim3(256), 0, st, a, hyp, H,
                       W, N, NP, cvol);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (bits + P2 <= 255)
        return dense_dispatch<uint8_t>(a, lines, H, W, N, NP, P1, P2, cvol, Lbuf, st);
    return dense_dispatch<uint16_t>(a, lines, H, W, N, NP, P1, P2, cvol, Lbuf, st);
}

hipError_t launch_sgm_bounded(const SgmBounded& a, int H, int W, int N, int P1, int P2,
                              int npaths, void* scratch, hipStream_t st) {
    const Lines lines = make_lines(H, W, npaths);
    const size_t dir_stride = (size_t)H * W * N;     // worst-case cells per direction
    const int HW = H * W;
    PixMeta* meta = (PixMeta*)scratch;
    uint16_t* Lbuf = (uint16_t*)((char*)scratch + ((size_t)HW * sizeof(PixMeta) + 255) / 256 * 256);
    hipLaunchKernelGGL(pix_meta_kernel, dim3((HW + 255) / 256), dim3(256), 0, st, a.off, a.lo, a.hi,
                       HW, meta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch ((N + 63) / 64) {
        case 1: e = bounded_launch<1>(a, meta, lines, H, W, P1, P2, dir_stride, Lbuf, st); break;
        case 2: e = bounded_launch<2>(a, meta, lines, H, W, P1, P2, dir_stride, Lbuf, st); break;
        case 3: e = bounded_launch<3>(a, meta, lines, H, W, P1, P2, dir_stride, Lbuf, st); break;
        default: e = bounded_launch<4>(a, meta, lines, H, W, P1, P2, dir_stride, Lbuf, st); break;
    }
    if (e != hipSuccess) return e;
    const int blocks = 2048;
    const int64_t* total = a.off + (int64_t)H * W;
    if (a.sum_bits == 16)
        hipLaunchKernelGGL(bounded_sum_kernel<uint16_t>, dim3(blocks), dim3(256), 0, st, Lbuf,
                           npaths, dir_stride, total, (uint16_t*)a.csum);
    else
        hipLaunchKernelGGL(bounded_sum_kernel<uint32_t>, dim3(blocks), dim3(256), 0, st, Lbuf,
                           npaths, dir_stride, total, (uint32_t*)a.csum);
    return hipGetLastError();
}

}  // namespace lf
