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
//     the next D steps in flight (D is a tuning parameter);
//   - the neighbours k-1 / k+1 of the previous pixel come from the lane's own
//     registers or, at the lane boundary, from lane l-1 / l+1 by a DPP wave
//     shift (wave_shr:1 / wave_shl:1);
//   - m = min_k L_r(p-r, k) is a DPP reduction (quad perms, half/row mirror, row
//     broadcasts) and a readlane, so it is wave-uniform in an SGPR.
// The initial stage stages each step's path-cost row in LDS and copies D rows
// at a time out with 16-byte stores.
// Path costs use the normalised recurrence (subtract m), which keeps them in
// [0, C + P2]: 8 bits suffice for the Census stage when bits + P2 <= 255.
// Hypotheses outside a pixel's range hold +inf (kInf) so they never win a min.
#include "lf_internal.h"

#include <algorithm>
#include <climits>
#include <type_traits>

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

// Path directions (du, dv): the 8 axis and diagonal neighbours, then the 8
// knight moves of the 16-path setting (Sec. 4.3).
const int kDirs[16][2] = {{1, 0},  {-1, 0},  {0, 1},  {0, -1}, {1, 1},  {-1, -1},
                          {1, -1}, {-1, 1},  {1, 2},  {-1, -2}, {2, 1},  {-2, -1},
                          {2, -1}, {-2, 1},  {1, -2}, {-1, 2}};
constexpr int kMaxPaths = 16;

// A path starts at every pixel whose predecessor p - r lies outside the image:
// the |dv| rows and |du| columns on the entry sides.
__host__ __device__ inline int num_lines(int H, int W, int du, int dv) {
    const int su = min(abs(du), W), sv = min(abs(dv), H);
    return sv * W + su * (H - sv);
}

// Lines of every direction, numbered consecutively: direction r owns global
// lines [base[r], base[r+1]); nlines = base[npaths].
struct Lines {
    int base[kMaxPaths + 1];
    int8_t du[kMaxPaths], dv[kMaxPaths];
    int npaths, nlines;
};

Lines make_lines(int H, int W, int npaths) {
    Lines L{};
    L.npaths = npaths;
    L.base[0] = 0;
    for (int r = 0; r < npaths; ++r) {
        L.du[r] = (int8_t)kDirs[r][0];
        L.dv[r] = (int8_t)kDirs[r][1];
        L.base[r + 1] = L.base[r] + num_lines(H, W, L.du[r], L.dv[r]);
    }
    L.nlines = L.base[npaths];
    return L;
}

struct LineInfo {
    int r, u0, v0, du, dv, len;
};

// Start pixel and length of global line g (wave-uniform; scalar arithmetic).
// Lines of a direction are the entry rows first (row-major), then the entry
// columns below / above them.
__device__ __forceinline__ LineInfo locate(const Lines& L, int H, int W, int g) {
    LineInfo li;
    // the direction of line g and its fields, read with constant indices only (the
    // argument record stays in registers)
    int r = 0, lbase = 0, du = L.du[0], dv = L.dv[0];
#pragma unroll
    for (int i = 1; i < kMaxPaths; ++i)
        if (i < L.npaths && g >= L.base[i]) {
            r = i;
            lbase = L.base[i];
            du = L.du[i];
            dv = L.dv[i];
        }
    const int line = g - lbase;
    const int su = min(abs(du), W), sv = min(abs(dv), H);
    li.r = r;
    li.du = du;
    li.dv = dv;
    if (line < sv * W) {                 // an entry row
        const int j = line / W;
        li.u0 = line - j * W;
        li.v0 = dv >= 0 ? j : H - 1 - j;
    } else {                             // an entry column, below/above the entry rows
        const int l2 = line - sv * W;
        const int i = l2 / su, j = l2 - i * su;
        li.u0 = du >= 0 ? j : W - 1 - j;
        li.v0 = dv >= 0 ? sv + i : H - 1 - sv - i;
    }
    const int lu = du > 0 ? (W - 1 - li.u0) / du + 1 : du < 0 ? li.u0 / -du + 1 : INT_MAX;
    const int lv = dv > 0 ? (H - 1 - li.v0) / dv + 1 : dv < 0 ? li.v0 / -dv + 1 : INT_MAX;
    li.len = min(lu, lv);
    return li;
}

// Work units of the path kernels with one line per wave.  Besides |W - H| + 1
// lines of length M = min(H, W), a diagonal direction (|du| = |dv| = 1) has one
// line of each length 1 .. M - 1 among its entry-row lines and one among its
// entry-column lines.  Its units are the full lines alone and the pairs of
// lengths m and M - m, run one after the other: every unit is M steps long, so
// all the waves of the launch have the same work and none is left running
// alone at the end.  Any other direction has one unit per line.
__host__ __device__ inline bool paired_dir(int du, int dv) {
    return (du == 1 || du == -1) && (dv == 1 || dv == -1);
}

__host__ __device__ inline int num_units(int H, int W, int du, int dv) {
    return paired_dir(du, dv) ? max(H, W) : num_lines(H, W, du, dv);
}

struct Units {
    int base[kMaxPaths + 1];       // direction r owns units [base[r], base[r+1])
    int nunits;
};

Units make_units(const Lines& L, int H, int W) {
    Units U{};
    for (int r = 0; r < L.npaths; ++r)
        U.base[r + 1] = U.base[r] + num_units(H, W, L.du[r], L.dv[r]);
    U.nunits = U.base[L.npaths];
    return U;
}

// The global lines of unit u (wave-uniform): line[0], and line[1] or -1.  In a
// diagonal direction, entry-row line j is min(W - j', H) long, j' = j for du > 0
// and W - 1 - j for du < 0, and entry-column line i (index W + i within the
// direction) min(W, H - 1 - i).
__device__ __forceinline__ void unit_lines(const Lines& L, const Units& U, int H, int W, int u,
                                           int (&line)[2]) {
    int r = 0, ub = 0, lb = 0, du = L.du[0], dv = L.dv[0];
#pragma unroll
    for (int i = 1; i < kMaxPaths; ++i)    // constant indices: the record stays in registers
        if (i < L.npaths && u >= U.base[i]) {
            r = i;
            ub = U.base[i];
            lb = L.base[i];
            du = L.du[i];
            dv = L.dv[i];
        }
    const int x = u - ub;
    int first = x, second = -1;
    if (paired_dir(du, dv)) {
        if (x < W && du < 0) first = W - 1 - x;        // the row line of length min(W - x, H)
        if (W >= H) {
            if (x > W - H) second = 2 * W - 1 - x;      // lengths W - x and H - (W - x)
        } else if (x >= 1 && x < W) {
            second = W + H - 1 - x;                    // lengths W - x and x
        }                                              // x >= W: a full column line
    }
    line[0] = lb + first;
    line[1] = second < 0 ? -1 : lb + second;
}

constexpr int kWavesPerBlock = 4;

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

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
    // X = Lp + P1 first: each DPP neighbour move then fuses into the min that
    // consumes it, and (for K = 2) none of the sources needs a copy
    uint32_t X[K];
#pragma unroll
    for (int j = 0; j < K; ++j) X[j] = Lp[j] + P1;
    const uint32_t left = dpp<0x138>(UINT_MAX, X[K - 1]);    // wave_shr:1 -> from lane l-1
    const uint32_t right = dpp<0x130>(UINT_MAX, X[0]);       // wave_shl:1 -> from lane l+1
    const uint32_t mP2 = m + P2;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint32_t lm = j == 0 ? left : X[j - 1];
        const uint32_t lp = j == K - 1 ? right : X[j + 1];
        const uint32_t t = min(min(Lp[j], mP2), min(lm, lp));
        L[j] = t + (C[j] - m);               // the cost byte less m: one SDWA subtract
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
// Initial stage, Eq. (7): the Census cost volume C[z][p][NPc] (8-bit; NPc = N + 2
// rounded up to 4, at most 256) of every cross view, computed once and read by
// all path directions.  Bytes k >= N of a row hold 255.  A workgroup builds the tile of 64 consecutive pixels x NP
// hypotheses in LDS with lanes over pixels -- for a fixed hypothesis the 64
// gathered Census strings are consecutive in memory for both shift axes -- and
// then writes the tile, which is contiguous in C, with 32-bit stores.
constexpr int kTilePix = 64;

struct CcvArgs {
    gptr<const uint64_t> cref;     // [C][H*W]
    gptr<const uint64_t> cview;    // [nv][C][H*W]
    gptr<const float> hyp;
    uint64_t cs4, ct4;        // s_hat - s, t_hat - t of cross view z in bits 16z..16z+15
                              // (int16; packed so that the record is never indexed)
    int nv, C, H, W, N, NP;   // NP: the row stride NPc
    uint32_t tiles;           // pixel tiles per view
    gptr<uint8_t> cvol;            // [nv][H*W][NPc]
};

__device__ __forceinline__ void ccv_block(const CcvArgs& a, uint32_t b, uint32_t* tile,
                                          int* s_sh) {
    const int z = (int)(b / a.tiles);
    const uint32_t t = b - (uint32_t)z * a.tiles;
    const int H = a.H, W = a.W, N = a.N, NP = a.NP;
    const uint32_t HW = (uint32_t)H * W;
    const uint32_t p0 = t * kTilePix;
    const int npix = (int)min((uint32_t)kTilePix, HW - p0);
    const int csz = (int16_t)(a.cs4 >> (16 * z)), ctz = (int16_t)(a.ct4 >> (16 * z));
    const bool along_u = ctz == 0;
    const int cs = along_u ? csz : ctz;
    for (int k = threadIdx.x; k < NP; k += 256)
        s_sh[k] = (int)rintf((float)cs * a.hyp[min(k, N - 1)]);
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t p = p0 + (uint32_t)min(lane, npix - 1);
    const int v = (int)(p / W), u = (int)(p - (uint32_t)v * W);
    // colour: one Census string per channel, Hamming distances summed (<= 3*64)
    const int C = a.C;
    uint64_t r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = c < C ? a.cref[(size_t)c * HW + p] : 0;
    const uint64_t* __restrict__ cv = a.cview + (size_t)z * C * HW;
    // The rounded shift is monotone in k, so consecutive hypotheses mostly share
    // it (at |s_hat - s| * (d_k+1 - d_k) < 1 a shift spans several k): wave w
    // walks its quarter of the row's 4-hypothesis words in order, gathers and
    // counts a Census string only when the shift changes, and writes each word
    // of four costs (255 past N) with one LDS store.
    const int NW = NP / 4;
    const int wb = NW * wave / 4, we = NW * (wave + 1) / 4;
    int prev = INT_MIN;
    uint32_t hd = 0;
    for (int w4 = wb; w4 < we; ++w4) {               // w4 is wave-uniform
        const int4 sh4 = *(const int4*)(s_sh + 4 * w4);
        const int shq[4] = {sh4.x, sh4.y, sh4.z, sh4.w};
        uint32_t word = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t val = 255;
            if (4 * w4 + q < N) {
                const int sh = __builtin_amdgcn_readfirstlane(shq[q]);
                if (sh != prev) {
                    prev = sh;
                    const uint32_t qq = along_u ? (uint32_t)(v * W + clampi(u + sh, 0, W - 1))
                                                : (uint32_t)(clampi(v + sh, 0, H - 1) * W + u);
                    hd = 0;
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        if (c < C) hd += (uint32_t)__popcll(r[c] ^ cv[(size_t)c * HW + qq]);
                }
                val = hd;
            }
            word |= val << (8 * q);
        }
        tile[lane * NW + w4] = word;
    }
    __syncthreads();
    // the tile is npix * NP contiguous bytes of C (NP is a multiple of 4): 16-byte
    // stores (4-byte aligned), then the last words one by one
    uint32_t* dst = (uint32_t*)(a.cvol + ((size_t)z * HW + p0) * NP);
    const int words = npix * NP / 4, quads = words / 4;
    for (int i = threadIdx.x; i < quads; i += 256) {
        uint4 q;
        __builtin_memcpy(&q, __builtin_assume_aligned(tile + 4 * i, 16), 16);
        __builtin_memcpy(dst + 4 * i, &q, 16);
    }
    for (int i = 4 * quads + threadIdx.x; i < words; i += 256) dst[i] = tile[i];
}

template <class Src>
__global__ __launch_bounds__(256) void census_cost_volume_kernel(Src src) {
    __shared__ __align__(16) uint32_t tile[kTilePix * LF_MAX_HYPOTHESES / 4];
    __shared__ __align__(16) int s_sh[LF_MAX_HYPOTHESES];
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const CcvArgs& a = member(src, vb, b);
        __syncthreads();                          // LDS of the previous block is read
        ccv_block(a, b, tile, s_sh);
    }
}

// SGM over the Census cost volume, every direction of every view in one launch.
// Output: Lbuf[r][z][p][NP], storage type LT, NP a multiple of 4 elements.
struct DenseArgs {
    gptr<const uint8_t> cvol;      // [nv][H*W][NPc]
    gptr<void> Lbuf;
    Lines lines;
    Units units;
    int nv, H, W, N, NP, NPc;
    uint32_t P1, P2;
    uint32_t wblocks;         // blocks per view
};

// Staged bytes per step of the initial path kernel: the lanes' 64 K path costs,
// rounded up to whole 128-byte lines, as are the rows in memory (a path-cost
// row of NP elements is never longer: see dense_lnp).
constexpr int dense_stage_row(int K, int elem_bytes) {
    return (64 * K * elem_bytes + 127) / 128 * 128;
}

// The K path costs of a lane, written as LT into the wave's staging row.
template <int K, typename LT>
__device__ __forceinline__ void stage_put(uint8_t* dst, const uint32_t (&L)[K]) {
    if constexpr (sizeof(LT) == 1) {
        if constexpr (K == 1) {
            *dst = (uint8_t)L[0];
        } else if constexpr (K == 2) {
            *(uint16_t*)dst = (uint16_t)((L[0] & 0xFFu) | (L[1] << 8));
        } else if constexpr (K == 4) {
            *(uint32_t*)dst = (L[0] & 0xFFu) | ((L[1] & 0xFFu) << 8) | ((L[2] & 0xFFu) << 16) |
                              (L[3] << 24);
        } else {
#pragma unroll
            for (int j = 0; j < K; ++j) dst[j] = (uint8_t)L[j];
        }
    } else {
        if constexpr (K == 1) {
            *(uint16_t*)dst = (uint16_t)L[0];
        } else if constexpr (K == 2) {
            *(uint32_t*)dst = (L[0] & 0xFFFFu) | (L[1] << 16);
        } else if constexpr (K == 4) {
            *(uint2*)dst = make_uint2((L[0] & 0xFFFFu) | (L[1] << 16),
                                      (L[2] & 0xFFFFu) | (L[3] << 16));
        } else {
#pragma unroll
            for (int j = 0; j < K; ++j) ((uint16_t*)dst)[j] = (uint16_t)L[j];
        }
    }
}

// kPad (8-bit path costs, K <= 2, and B + 2 P2 <= 255 + P1 for the largest Census
// cost B): hypotheses k >= N read the 255 that pads each cost row instead of
// adding kInf.  Their path costs then stay >= 255 while every real one stays
// <= B + P2 <= 255, so they never lower the minimum m, and as the neighbour of
// k = N-1 their 255 + P1 >= m + P2 (m <= B + P2) never wins the min of Eq. (8):
// the real path costs are those of the exact recurrence.
//
// Stores.  A path-cost row (NP elements) per step would be one narrow store per
// step, and those stores took about a third of the kernel's vector-memory
// issue.  Instead each step's row goes to the wave's staging area in LDS, and
// after every D steps the wave copies the D rows out with 16-byte stores, the
// lanes over (row, 16-byte chunk) pairs, and one store for the rows' short
// tails: 16 rows of 100 bytes are three store instructions.  Row elements
// k >= N hold don't-care values.
template <int K, typename LT, int D, bool kPad>
__device__ __forceinline__ void dense_line(const DenseArgs& a, int z, const LineInfo& li,
                                           uint8_t* wst) {
    constexpr int kRow = dense_stage_row(K, sizeof(LT));    // staged bytes per step
    constexpr int kRounds = (D * kRow / 16 + 63) / 64;      // 16-byte copies per lane
    const int lane = threadIdx.x & 63;
    const int H = a.H, W = a.W, N = a.N, NPc = a.NPc;
    const uint32_t P1 = a.P1, P2 = a.P2;
    const uint32_t HW = (uint32_t)H * W;
    const uint8_t* __restrict__ cz = a.cvol + (size_t)z * HW * NPc;
    const int rb = a.NP * (int)sizeof(LT);                  // bytes per path-cost row
    uint8_t* __restrict__ out = (uint8_t*)a.Lbuf + ((size_t)li.r * a.nv + z) * HW * rb;

    // Copy plan of a flush, fixed per line.  A row is c16 whole 16-byte chunks
    // and a tail of 0, 4, 8 or 12 bytes (rows are 4-byte aligned).  Copy j of
    // this lane moves chunk c of staged row s to byte goff[j] past the flush's
    // base address, that of the lowest-addressed row (rows follow the line, so
    // for a direction running backwards it is the block's last row); lane s < D
    // also moves the tail of row s.  Chunks past the D rows repeat the last one
    // (the same bytes to the same place).
    const int c16 = rb >> 4, tail = rb & 15, nchunk = D * c16;
    const int dstep = li.dv * W + li.du;                    // pixels per step
    const int sbytes = dstep * rb;
    const int minoff = min(0, (D - 1) * sbytes);
    uint32_t loff[kRounds], goff[kRounds];
    int srow[kRounds];
#pragma unroll
    for (int j = 0; j < kRounds; ++j) {
        const int idx = min(lane + 64 * j, max(nchunk - 1, 0));
        const int s = c16 ? idx / c16 : 0, c = idx - s * c16;
        srow[j] = s;
        loff[j] = (uint32_t)(s * kRow + c * 16);
        goff[j] = (uint32_t)(s * sbytes - minoff + c * 16);
    }
    const int tsrow = min(lane, D - 1);
    const uint32_t tloff = (uint32_t)(tsrow * kRow + c16 * 16);
    const uint32_t tgoff = (uint32_t)(tsrow * sbytes - minoff + c16 * 16);

    // the lane's K bytes of a pixel row; lanes past N read the row's last bytes
    // (with kPad: its 255 padding, since NPc >= N + 2) and, without kPad, add kInf
    const uint32_t lofs = (uint32_t)min(lane * K, NPc - K);
    uint32_t cinit[K];
#pragma unroll
    for (int j = 0; j < K; ++j) cinit[j] = kPad || lane * K + j < N ? 0u : kInf;
    const int last = li.len - 1;
    const int64_t srow_bytes = (int64_t)dstep * NPc;       // cost-row bytes per step
    // One load per step for the K bytes.  The loads of a block of D steps go
    // through a buffer descriptor based at the lowest-addressed row among them;
    // a step's row offset from it (>= 0, < 2^31) is the scalar offset, the lane's
    // byte within the row the vector offset: no per-step vector arithmetic.
    auto block_rsrc = [&](int nb, int& lo) {
        lo = dstep >= 0 ? min(nb, last) : min(nb + D - 1, last);
        const uint32_t p = (uint32_t)((li.v0 + lo * li.dv) * W + li.u0 + lo * li.du);
        return __builtin_amdgcn_make_buffer_rsrc((void*)(cz + (size_t)p * NPc), (short)0,
                                                 0x7FFFFFFF, 0x00020000);
    };
    auto load = [&](__amdgpu_buffer_rsrc_t rs, int lo, int step) -> uint32_t {
        const int so = (int)((int64_t)(min(step, last) - lo) * srow_bytes);
        if constexpr (K == 1) {
            return __builtin_amdgcn_raw_buffer_load_b8(rs, lofs, so, 0);
        } else if constexpr (K == 2) {
            return __builtin_amdgcn_raw_buffer_load_b16(rs, lofs, so, 0);
        } else if constexpr (K == 4) {
            return __builtin_amdgcn_raw_buffer_load_b32(rs, lofs, so, 0);
        } else {
            return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, lofs, so, 0) |
                   ((uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, lofs + 1, so, 0) << 8) |
                   ((uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, lofs + 2, so, 0) << 16);
        }
    };
    uint32_t cb[D];
    {
        int lo;
        const __amdgpu_buffer_rsrc_t rs = block_rsrc(0, lo);
#pragma unroll
        for (int i = 0; i < D; ++i) cb[i] = load(rs, lo, i);
    }

    uint8_t* const mine = wst + lane * K * (int)sizeof(LT);
    uint32_t Lp[K], m = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) Lp[j] = kInf;
    for (int base = 0; base < li.len; base += D) {
        int lo;
        const __amdgpu_buffer_rsrc_t rs = block_rsrc(base + D, lo);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int step = base + i;           // steps past the line end are computed
            uint32_t C[K];                       // and not copied out
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const uint32_t byte = (cb[i] >> (8 * j)) & 0xFFu;
                C[j] = kPad ? byte : byte + cinit[j];
            }
            cb[i] = load(rs, lo, step + D);      // refill the slot just consumed
            uint32_t L[K];
            if (step == 0) {
#pragma unroll
                for (int j = 0; j < K; ++j) L[j] = C[j];
            } else {
                sgm_step<K>(Lp, m, P1, P2, C, L);
            }
            m = wave_min(lane_min(L));
            stage_put<K, LT>(mine + i * kRow, L);
#pragma unroll
            for (int j = 0; j < K; ++j) Lp[j] = L[j];
        }
        // flush: the staged rows were written by other lanes of this wave, whose
        // LDS accesses complete in order
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int rows = min(D, li.len - base);
        const uint32_t pb = (uint32_t)((li.v0 + base * li.dv) * W + li.u0 + base * li.du);
        uint8_t* const ob = out + (int64_t)pb * rb + minoff;
        const bool stream = (rb & 127) == 0;     // whole-line rows
        // LDS offsets are 16-byte aligned; rows in memory 4-byte aligned
        auto copy = [&](uint32_t lo, uint32_t go, auto n) {
            constexpr int kBytes = decltype(n)::value;
            using V = typename std::conditional<kBytes == 16, uint4,
                      typename std::conditional<kBytes == 12, uint3,
                      typename std::conditional<kBytes == 8, uint2, uint32_t>::type>::type>::type;
            V v;
            __builtin_memcpy(&v, __builtin_assume_aligned(wst + lo, 16), kBytes);
            if constexpr (kBytes == 16) {
                if (stream) {
                    // rows are whole cache lines, read once by the sum: streaming
                    // (non-temporal) stores, measured 0.33 vs 0.41 ms for the kernel
                    uint32_t* d = (uint32_t*)__builtin_assume_aligned(ob + go, 16);
                    __builtin_nontemporal_store(v.x, d);
                    __builtin_nontemporal_store(v.y, d + 1);
                    __builtin_nontemporal_store(v.z, d + 2);
                    __builtin_nontemporal_store(v.w, d + 3);
                    return;
                }
            }
            __builtin_memcpy(__builtin_assume_aligned(ob + go, 4), &v, kBytes);
        };
#pragma unroll
        for (int j = 0; j < kRounds; ++j) {
            if (64 * j >= nchunk) break;         // wave-uniform
            if (rows == D || srow[j] < rows) copy(loff[j], goff[j], std::integral_constant<int, 16>());
        }
        if (tail && tsrow < rows) {
            if (tail == 4) copy(tloff, tgoff, std::integral_constant<int, 4>());
            else if (tail == 8) copy(tloff, tgoff, std::integral_constant<int, 8>());
            else copy(tloff, tgoff, std::integral_constant<int, 12>());
        }
        // the next steps overwrite the staging rows only after these reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <class Src, int K, typename LT, int D, bool kPad>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sgm_dense_paths_kernel(Src src) {
    constexpr int kWaveBytes = D * dense_stage_row(K, sizeof(LT));
    __shared__ __align__(16) uint8_t stage[kWavesPerBlock * kWaveBytes];
    uint8_t* const wst = stage + (threadIdx.x >> 6) * kWaveBytes;
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const DenseArgs& a = member(src, vb, b);
        const int z = (int)(b / a.wblocks);               // the view
        const uint32_t wb = b - (uint32_t)z * a.wblocks;
        const int u = __builtin_amdgcn_readfirstlane(wb * kWavesPerBlock + (threadIdx.x >> 6));
        if (u >= a.units.nunits) continue;                // wave-uniform
        int line[2];
        unit_lines(a.lines, a.units, a.H, a.W, u, line);
        for (int part = 0; part < 2; ++part) {            // one copy of the line loop
            if (line[part] < 0) break;
            dense_line<K, LT, D, kPad>(a, z, locate(a.lines, a.H, a.W, line[part]), wst);
        }
    }
}

// Sum over directions + WTA (Eq. 9-10) of the initial stage: one wave per pixel,
// lane l holds hypotheses 2l and 2l+1 (+128 per round); lowest index on ties.
struct SumWtaArgs {
    gptr<const void> Lbuf;
    int64_t HW;
    int nv, N, NP;
    gptr<int16_t> dmap;            // [nv][H*W]
};

template <typename LT, int kPaths>
__device__ __forceinline__ void sum_wta_block(const SumWtaArgs& a, uint32_t b) {
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)b * 4 + (threadIdx.x >> 6);       // q = z*HW + p
    if (q >= a.nv * a.HW) return;                                 // wave-uniform
    const int N = a.N, NP = a.NP;
    const size_t dir_stride = (size_t)a.nv * a.HW * NP;
    const LT* __restrict__ base = (const LT*)a.Lbuf + (size_t)q * NP;
    uint32_t key = UINT_MAX;
    for (int k = 2 * lane; k < N; k += 128) {
        uint32_t x[kPaths];                                       // all loads in flight first
#pragma unroll
        for (int r = 0; r < kPaths; ++r) {
            const LT* e = base + (size_t)r * dir_stride + k;
            if constexpr (sizeof(LT) == 1) x[r] = __builtin_nontemporal_load((const uint16_t*)e);
            else x[r] = __builtin_nontemporal_load((const uint32_t*)e);
        }
        uint32_t t0 = 0, t1 = 0;
#pragma unroll
        for (int r = 0; r < kPaths; ++r) {
            if constexpr (sizeof(LT) == 1) {
                t0 += x[r] & 0xFF;
                t1 += x[r] >> 8;
            } else {
                t0 += x[r] & 0xFFFF;
                t1 += x[r] >> 16;
            }
        }
        key = min(key, (t0 << 8) | (uint32_t)k);
        if (k + 1 < N) key = min(key, (t1 << 8) | (uint32_t)(k + 1));
    }
    key = wave_min(key);
    if (lane == 0) a.dmap[q] = (int16_t)(key & 0xFF);
}

// The same for 8-bit path costs with rows of at most 128 bytes (N <= 128): a
// row of 16 lanes per pixel, 8 bytes (8 hypotheses) per lane, so one 64-lane
// load reads four pixels' rows of a direction (512 bytes).  The sums are kept
// two per register in 16-bit fields (at most 16 * 255 per field: no carry
// between fields); the argmin is a DPP minimum within the row of 16 lanes.
// Lanes past a row's end read the next row (or the slack after the volume) and
// drop those hypotheses (k >= N).
template <int kPaths>
__device__ __forceinline__ void sum_wta_rows_block(const SumWtaArgs& a, uint32_t b) {
    const int sub = threadIdx.x & 15;
    const int64_t nq = a.nv * a.HW;
    const int64_t q = (int64_t)b * 16 + (threadIdx.x >> 4);       // this row's pixel
    const int64_t qq = q < nq ? q : nq - 1;                        // rows past the end
    const int N = a.N;                                             // load in bounds
    const size_t dir_stride = (size_t)a.nv * a.HW * a.NP;
    const uint8_t* __restrict__ base = (const uint8_t*)a.Lbuf + (size_t)qq * a.NP + sub * 8;
    // the path costs are read once: non-temporal loads (measured 0.155 vs 0.204
    // ms at the benchmark size) keep them from displacing what L2 holds
    uint32_t x0[kPaths], x1[kPaths];
#pragma unroll
    for (int r = 0; r < kPaths; ++r) {
        const uint32_t* pp = (const uint32_t*)(base + (size_t)r * dir_stride);
        x0[r] = __builtin_nontemporal_load(pp);
        x1[r] = __builtin_nontemporal_load(pp + 1);
    }
    // acc[0]: bytes 0, 2; acc[1]: 1, 3; acc[2]: 4, 6; acc[3]: 5, 7 (low, high field)
    uint32_t acc[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int r = 0; r < kPaths; ++r) {
        acc[0] += x0[r] & 0x00FF00FFu;
        acc[1] += (x0[r] >> 8) & 0x00FF00FFu;
        acc[2] += x1[r] & 0x00FF00FFu;
        acc[3] += (x1[r] >> 8) & 0x00FF00FFu;
    }
    uint32_t key = UINT_MAX;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t t = (acc[(i >> 2) * 2 + (i & 1)] >> (16 * ((i >> 1) & 1))) & 0xFFFFu;
        const int k = sub * 8 + i;
        if (k < N) key = min(key, (t << 8) | (uint32_t)k);
    }
    key = min(key, dpp<0xB1>(UINT_MAX, key));     // quad_perm [1,0,3,2]
    key = min(key, dpp<0x4E>(UINT_MAX, key));     // quad_perm [2,3,0,1]
    key = min(key, dpp<0x141>(UINT_MAX, key));    // row_half_mirror
    key = min(key, dpp<0x140>(UINT_MAX, key));    // row_mirror: the row's minimum
    if (sub == 0 && q < nq) a.dmap[q] = (int16_t)(key & 0xFF);
}

template <class Src, int kPaths>
__global__ __launch_bounds__(256) void dense_sum_wta_rows_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const SumWtaArgs& a = member(src, vb, b);
        sum_wta_rows_block<kPaths>(a, b);
    }
}

template <class Src, typename LT, int kPaths>
__global__ __launch_bounds__(256) void dense_sum_wta_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const SumWtaArgs& a = member(src, vb, b);
        sum_wta_block<LT, kPaths>(a, b);
    }
}

// Optional outputs of the initial stage for checking: the Census cost of Eq. (7)
// and the aggregated cost of Eq. (9) of every cross view, [nv][H*W][N], copied
// and summed out of the stage's own buffers (element e = (z*HW + p)*N + k).
struct ExportArgs {
    gptr<const void> src;          // cvol [nv][HW][NPc] (8-bit), or Lbuf [npaths][nv][HW][NP]
    gptr<void> dst;                // [nv][HW][N]: 8-bit costs, or 16-bit sums
    int64_t rows;             // nv * HW
    int N, NP, npaths, lt;    // lt: bytes per path-cost element (sums)
};

template <class Src, bool kSum>
__global__ __launch_bounds__(256) void initial_export_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const ExportArgs& a = member(src, vb, b);
        const int64_t e = (int64_t)b * 256 + threadIdx.x;
        if (e >= a.rows * a.N) continue;
        const int64_t q = e / a.N;
        const int64_t at = q * a.NP + (e - q * a.N);
        if constexpr (!kSum) {
            ((uint8_t*)a.dst)[e] = ((const uint8_t*)a.src)[at];
        } else {
            const int64_t dir = a.rows * a.NP;
            uint32_t s = 0;
            for (int r = 0; r < a.npaths; ++r)
                s += a.lt == 1 ? ((const uint8_t*)a.src)[r * dir + at]
                               : ((const uint16_t*)a.src)[r * dir + at];
            ((uint16_t*)a.dst)[e] = (uint16_t)s;
        }
    }
}

// ---------------------------------------------------------------------------
// Final stage: CSR volume over per-pixel ranges [lo, hi].  Output Lbuf[r][cell].
// meta[p] = {q = off[p] - lo[p] + N (int64, low half first), lo | hi << 16}: one
// 16-byte load per step, or one 8-byte load of the first two words where 32-bit
// offsets suffice.  Cell k of pixel p is q + k - N; q + k itself is positive for
// every k >= 0 (off[p] >= 0, lo[p] < N), so it can serve as an unsigned offset
// from N cells before the volume.
struct alignas(16) PixMeta {
    uint32_t q_lo;
    int32_t lohi;
    uint32_t q_hi;
    int32_t pad;
    __device__ int64_t base(int N) const {   // off - lo
        return (int64_t)(((uint64_t)q_hi << 32) | q_lo) - N;
    }
};

struct MetaArgs {
    gptr<const int64_t> off;
    gptr<const int16_t> lo;
    gptr<const int16_t> hi;
    gptr<PixMeta> meta;
    int HW, N;
};

template <class Src>
__global__ __launch_bounds__(256) void pix_meta_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const MetaArgs& a = member(src, vb, b);
        const int p = (int)b * 256 + threadIdx.x;
        if (p >= a.HW) continue;
        // bounds outside the documented 0 <= lo <= hi < N are clamped into it; that
        // only narrows a range, so its cells stay within the pixel's own
        const int lo = clampi(a.lo[p], 0, a.N - 1), hi = clampi(a.hi[p], lo, a.N - 1);
        PixMeta m;
        const uint64_t q = (uint64_t)(a.off[p] - lo + a.N);
        m.q_lo = (uint32_t)q;
        m.lohi = (int32_t)((uint32_t)lo | ((uint32_t)hi << 16));
        m.q_hi = (uint32_t)(q >> 32);
        m.pad = 0;
        a.meta[p] = m;
    }
}

struct BoundedArgs {
    gptr<const uint16_t> cost;
    gptr<const PixMeta> meta;
    gptr<uint16_t> Lbuf;           // [npaths][dir_stride]
    size_t dir_stride;
    Lines lines;
    Units units;                   // of the 64-lane kernel (one line per wave)
    int H, W, N;
    uint32_t P1, P2;
};

template <int K, int D>
__device__ __forceinline__ void bounded_line(const BoundedArgs& a, const LineInfo& li) {
    constexpr int kMeta = D, kCost = D / 2;   // two-stage prefetch
    const int lane = threadIdx.x & 63;
    const int W = a.W;
    const uint32_t P1 = a.P1, P2 = a.P2;
    const uint16_t* __restrict__ cost = a.cost;
    const PixMeta* __restrict__ meta = a.meta;
    uint16_t* __restrict__ out = a.Lbuf + (size_t)li.r * a.dir_stride;

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
            c[j] = cost[pm.base(a.N) + k];
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
            // refill: costs for step + kCost (its meta arrived kMeta - kCost steps ago)
            load_cost(mb[(i + kCost) % kMeta], cb[i % kCost]);
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
                if (live && k >= lo && k <= hi) out[pm.base(a.N) + k] = (uint16_t)L[j];
            }
            // the slot's metadata for step + kMeta, loaded after the last use of
            // this step's (so the load can take the same registers: no copies,
            // which would wait for every load in flight, at the loop's back edge)
            mb[i] = load_meta(min(step + kMeta, li.len - 1));
#pragma unroll
            for (int j = 0; j < K; ++j) Lp[j] = L[j];
        }
    }
}

// The same line loop with the cost volume, the pixel metadata and this
// direction's path costs addressed through buffer descriptors, for volumes of
// less than 2^31 bytes: 32-bit byte offsets instead of 64-bit addresses.  A
// metadata load takes its pixel's offset as the scalar operand (no vector
// arithmetic), a cost gather med3(k, lo, hi) and one shift-add, and a step's
// stores one shift-add.  The descriptors start N cells before the volumes, so
// that the offsets q + k are never negative (the store of a lane whose first
// hypothesis lies below the range would otherwise start from a wrapped offset,
// and the hardware drops a store whose vector offset is out of range).  A lane's
// hypothesis k lies in [lo, hi] exactly when the clamp leaves it unchanged.
template <int K, int D>
__device__ __forceinline__ void bounded_line_buf(const BoundedArgs& a, const LineInfo& li) {
    constexpr int kMeta = D, kCost = D / 2;   // two-stage prefetch
    const int lane = threadIdx.x & 63;
    const int W = a.W;
    const uint32_t P1 = a.P1, P2 = a.P2;
    const int32_t vol_bytes = (int32_t)((a.dir_stride + a.N) * 2);
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const uint16_t*)a.cost - a.N), (short)0, vol_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rm = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(const PixMeta*)a.meta, (short)0, a.H * W * (int)sizeof(PixMeta), 0x00020000);
    const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((uint16_t*)a.Lbuf + (size_t)li.r * a.dir_stride - a.N), (short)0, vol_bytes,
        0x00020000);
    struct Meta {
        uint32_t base, lohi;       // low 32 bits of q; lo | hi << 16
    };
    auto load_meta = [&](int step) -> Meta {
        const int u = li.u0 + step * li.du, v = li.v0 + step * li.dv;
        const auto x = __builtin_amdgcn_raw_buffer_load_b64(
            rm, 0, (v * W + u) * (int)sizeof(PixMeta), 0);
        return Meta{x[0], x[1]};
    };
    int kl[K];                                 // the lane's hypotheses
#pragma unroll
    for (int j = 0; j < K; ++j) kl[j] = lane * K + j;
    // gather of the K costs of a pixel; hypotheses outside [lo, hi] read a cell
    // of the pixel and are replaced by kInf when used
    auto load_cost = [&](const Meta& pm, uint32_t (&c)[K]) {
        const int lo = (int)(pm.lohi & 0xFFFF), hi = (int)(pm.lohi >> 16);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t k = (uint32_t)min(max(kl[j], lo), hi);
            c[j] = __builtin_amdgcn_raw_buffer_load_b16(rc, (pm.base + k) << 1, 0, 0);
        }
    };
    Meta mb[kMeta];
    uint32_t cb[kCost][K];
#pragma unroll
    for (int i = 0; i < kMeta; ++i) mb[i] = load_meta(min(i, li.len - 1));
#pragma unroll
    for (int i = 0; i < kCost; ++i) load_cost(mb[i], cb[i]);

    uint32_t Lp[K], m = 0;                     // step 0 reduces to L = C
#pragma unroll
    for (int j = 0; j < K; ++j) Lp[j] = 0;
    for (int base = 0; base < li.len; base += kMeta) {
#pragma unroll
        for (int i = 0; i < kMeta; ++i) {
            const int step = base + i;           // steps past the line end are computed
            const Meta pm = mb[i];               // and not stored
            const int lo = (int)(pm.lohi & 0xFFFF), hi = (int)(pm.lohi >> 16);
            bool in[K];
            uint32_t C[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                in[j] = min(max(kl[j], lo), hi) == kl[j];
                C[j] = in[j] ? cb[i % kCost][j] : kInf;
            }
            load_cost(mb[(i + kCost) % kMeta], cb[i % kCost]);
            uint32_t L[K];
            sgm_step<K>(Lp, m, P1, P2, C, L);   // with Lp = 0 and m = 0: L = C at step 0
            m = wave_min(lane_min(L));
            const bool live = step < li.len;
            const uint32_t ob = (pm.base + (uint32_t)kl[0]) << 1;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (live && in[j])
                    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)L[j], ro, ob, 2 * j, 0);
            // the slot's metadata for step + kMeta, loaded after the last use of
            // this step's (so the load can take the same registers: no copies,
            // which would wait for every load in flight, at the loop's back edge)
            mb[i] = load_meta(min(step + kMeta, li.len - 1));
#pragma unroll
            for (int j = 0; j < K; ++j) Lp[j] = L[j];
        }
    }
}

template <class Src, int K, int D, bool kBuf>
__global__ __launch_bounds__(64 * kWavesPerBlock) void sgm_bounded_paths_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const BoundedArgs& a = member(src, vb, b);
        const int u = __builtin_amdgcn_readfirstlane(b * kWavesPerBlock + (threadIdx.x >> 6));
        if (u >= a.units.nunits) continue;            // wave-uniform
        int line[2];
        unit_lines(a.lines, a.units, a.H, a.W, u, line);
        for (int part = 0; part < 2; ++part) {        // one copy of the line loop
            if (line[part] < 0) break;
            if constexpr (kBuf)
                bounded_line_buf<K, D>(a, locate(a.lines, a.H, a.W, line[part]));
            else
                bounded_line<K, D>(a, locate(a.lines, a.H, a.W, line[part]));
        }
    }
}

// The bounded SGM with G lanes per path line (G = 16 or 32: 64/G lines per wave).
// Most pixels keep a window of 2*lambda+1 hypotheses, so one wave per line
// leaves most lanes idle; here a line's G lanes cover its pixel's range in
// chunks of G hypotheses (one chunk for a narrow window, ceil(N/G) for a
// full-range pixel), lane j of chunk c holding k = lo + G*c + j.
//
// A pixel's range need not overlap its predecessor's, so the previous path costs
// are kept by hypothesis index, not by lane: each line has two LDS rows of N + 2
// entries (k = -1 .. N), written on alternate steps.  An entry holds the path
// cost in its low 16 bits and the step that wrote it in the high 16 bits; at
// step s the predecessor's entries are those tagged s - 1, and subtracting
// (s-1) << 16 leaves their value while every other entry (older steps, never
// written) becomes >= 65536, which loses to m + P2 <= 65535 and does not wrap
// when P1 is added (path costs <= cap + P2 <= 65535 - P2).  So the terms of
// Eq. (8) outside R(p - r) are omitted without clearing anything.  m, the
// minimum over R(p - r), is the row minimum of the previous step's costs.
constexpr int kB16Waves = 4;                      // waves per workgroup

// Entries of one LDS row: N + 2, padded so that the rows of the lines of a wave
// (two per line) start on different banks.
__host__ __device__ constexpr int b16_row(int N) { return (N + 2 + 15) / 16 * 16 + 8; }

// Minimum over each group of G lanes (G = 16: a DPP row; 32: two rows), in
// every lane of the group.
template <int G>
__device__ __forceinline__ uint32_t group_min(uint32_t v) {
    v = min(v, dpp<0xB1>(UINT_MAX, v));           // quad_perm [1,0,3,2]
    v = min(v, dpp<0x4E>(UINT_MAX, v));           // quad_perm [2,3,0,1]
    v = min(v, dpp<0x141>(UINT_MAX, v));          // row_half_mirror
    v = min(v, dpp<0x140>(UINT_MAX, v));          // row_mirror: the row's minimum
    if constexpr (G == 32)                        // swap the rows of each 32-lane half
        v = min(v, (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F));
    return v;
}

template <int G, int KC, int DM, int DC>
__device__ __forceinline__ void bounded_group_wave(const BoundedArgs& a, uint32_t b,
                                                   uint32_t* lds) {
    constexpr int kLines = 64 / G;                // lines per wave
    const int lane = threadIdx.x & 63, sub = lane & (G - 1), grp = lane / G;
    const int wave = threadIdx.x >> 6;
    const int H = a.H, W = a.W, N = a.N;
    const uint32_t P1 = a.P1, P2 = a.P2;
    const int g = ((int)b * kB16Waves + wave) * kLines + grp;   // this group's line
    const int nlines = a.lines.nlines;
    LineInfo li{0, 0, 0, 0, 0, 0};
    if (g < nlines) li = locate(a.lines, H, W, g);
    // steps: the longest line of the wave (wave-uniform)
    int steps = 0;
#pragma unroll
    for (int i = 0; i < kLines; ++i) steps = max(steps, __builtin_amdgcn_readlane(li.len, i * G));
    if (steps == 0) return;
    const int RP = b16_row(N);
    uint32_t* const row0 = lds + (size_t)(wave * kLines + grp) * 2 * RP;
    for (int i = sub; i < 2 * RP; i += G) row0[i] = 0xFFFF0000u;     // no step wrote it
    const PixMeta* __restrict__ meta = a.meta;
    const uint16_t* __restrict__ cost = a.cost;
    uint16_t* __restrict__ out = a.Lbuf + (size_t)li.r * a.dir_stride;
    const int last = max(li.len - 1, 0);
    auto pix = [&](int step) {                    // steps past the line repeat its end
        const int st = min(step, last);
        return (uint32_t)((li.v0 + st * li.dv) * W + li.u0 + st * li.du);
    };
    PixMeta mb[DM];
    uint32_t cb[DC][KC];
    auto load_costs = [&](const PixMeta& pm, uint32_t (&c)[KC]) {
        const int lo = pm.lohi & 0xFFFF, hi = pm.lohi >> 16;
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int k = lo + G * j + sub;
            c[j] = k <= hi ? (uint32_t)cost[pm.base(N) + k] : 0u;
        }
    };
#pragma unroll
    for (int i = 0; i < DM; ++i) mb[i] = meta[in_vgpr(pix(i))];
#pragma unroll
    for (int i = 0; i < DC; ++i) load_costs(mb[i], cb[i]);

    uint32_t m = 0;
    for (int base = 0; base < steps; base += DM) {
#pragma unroll
        for (int i = 0; i < DM; ++i) {
            const int step = base + i;            // wave-uniform
            const PixMeta pm = mb[i];
            const int lo = pm.lohi & 0xFFFF, hi = pm.lohi >> 16;
            uint32_t C[KC];
#pragma unroll
            for (int j = 0; j < KC; ++j) C[j] = cb[i % DC][j];
            // refill: the costs of step + DC (its meta arrived DM - DC steps ago),
            // then the meta of step + DM
            load_costs(mb[(i + DC) % DM], cb[i % DC]);
            mb[i] = meta[in_vgpr(pix(step + DM))];
            const bool live = step < li.len;
            uint32_t* const prev = row0 + ((step + 1) & 1) * RP;    // written at step - 1
            uint32_t* const cur = row0 + (step & 1) * RP;
            const uint32_t tag = (uint32_t)(step - 1) << 16;
            const uint32_t mP2 = m + P2;
            uint32_t rmin = UINT_MAX;
#pragma unroll
            for (int j = 0; j < KC; ++j) {
                const int k = lo + G * j + sub;
                if (k <= hi) {
                    uint32_t L;
                    if (step == 0) {
                        L = C[j];
                    } else {
                        const uint32_t e0 = prev[k + 1] - tag;      // k
                        const uint32_t em = prev[k] - tag;          // k - 1
                        const uint32_t ep = prev[k + 2] - tag;      // k + 1
                        const uint32_t t = min(min(e0, min(em, ep) + P1), mP2);
                        L = t + C[j] - m;
                    }
                    cur[k + 1] = L | ((uint32_t)step << 16);
                    if (live) out[pm.base(N) + k] = (uint16_t)L;
                    rmin = min(rmin, L);
                }
            }
            m = group_min<G>(rmin);
            // the next step reads what the other lanes of this wave wrote
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

template <class Src, int G, int KC>
__global__ __launch_bounds__(64 * kB16Waves) void sgm_bounded_group_kernel(Src src) {
    __shared__ uint32_t lds[kB16Waves * (64 / G) * 2 * b16_row(KC * G)];
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const BoundedArgs& a = member(src, vb, b);
        __syncthreads();                          // the previous block's rows are done
        bounded_group_wave<G, KC, 8, 4>(a, b, lds);
    }
}

// csum[c] = sum_r Lbuf[r][c] over the cells of the CSR volume; each of a light
// field's nblk workgroups strides over its device-side cell count.
struct BsumArgs {
    gptr<const uint16_t> Lbuf;     // [npaths][dir_stride]
    size_t dir_stride;
    gptr<const int64_t> total;     // device-side cell count
    gptr<void> csum;
    uint32_t nblk;
};

template <class Src, typename SumT, int kPaths>
__global__ __launch_bounds__(256) void bounded_sum_kernel(Src src) {
    for (uint32_t vb = blockIdx.x; vb < src.total; vb += gridDim.x) {
        uint32_t b;
        const BsumArgs& a = member(src, vb, b);
        // the device-side count, never past the buffers (offsets that are not the
        // prefix sum of in-range widths would otherwise run past them)
        const int64_t n = min(*a.total, (int64_t)a.dir_stride);
        const uint16_t* __restrict__ L = a.Lbuf;
        SumT* __restrict__ csum = (SumT*)a.csum;
        for (int64_t c = (int64_t)b * 256 + threadIdx.x; c < n; c += (int64_t)a.nblk * 256) {
            uint32_t x[kPaths];
#pragma unroll
            for (int r = 0; r < kPaths; ++r)
                x[r] = __builtin_nontemporal_load(L + (size_t)r * a.dir_stride + c);
            uint32_t s = 0;
#pragma unroll
            for (int r = 0; r < kPaths; ++r) s += x[r];
            csum[c] = (SumT)s;
        }
    }
}

// --- host-side dispatch of the kernel variants ---------------------------------
template <int K, typename LT, bool kPad>
hipError_t dense_variant(Runner& r, const std::vector<DenseArgs>& args,
                         const std::vector<uint32_t>& blocks) {
    switch (r.tune.dense_depth) {
        case 4:
            return launch(r, kStInitPaths, sgm_dense_paths_kernel<Single<DenseArgs>, K, LT, 4, kPad>,
                          sgm_dense_paths_kernel<Group<DenseArgs>, K, LT, 4, kPad>, args, blocks,
                          64 * kWavesPerBlock);
        case 16:
            return launch(r, kStInitPaths, sgm_dense_paths_kernel<Single<DenseArgs>, K, LT, 16, kPad>,
                          sgm_dense_paths_kernel<Group<DenseArgs>, K, LT, 16, kPad>, args, blocks,
                          64 * kWavesPerBlock);
        default:
            return launch(r, kStInitPaths, sgm_dense_paths_kernel<Single<DenseArgs>, K, LT, 8, kPad>,
                          sgm_dense_paths_kernel<Group<DenseArgs>, K, LT, 8, kPad>, args, blocks,
                          64 * kWavesPerBlock);
    }
}

// v: 0 8-bit path costs, 1 16-bit, 2 8-bit with the padded rows standing in for
// kInf (K <= 2 only)
hipError_t dense_k(Runner& r, int K, int v, const std::vector<DenseArgs>& args,
                   const std::vector<uint32_t>& blocks) {
    if (v == 2) return K == 1 ? dense_variant<1, uint8_t, true>(r, args, blocks)
                              : dense_variant<2, uint8_t, true>(r, args, blocks);
    if (v == 1) {
        switch (K) {
            case 1: return dense_variant<1, uint16_t, false>(r, args, blocks);
            case 2: return dense_variant<2, uint16_t, false>(r, args, blocks);
            case 3: return dense_variant<3, uint16_t, false>(r, args, blocks);
            default: return dense_variant<4, uint16_t, false>(r, args, blocks);
        }
    }
    switch (K) {
        case 1: return dense_variant<1, uint8_t, false>(r, args, blocks);
        case 2: return dense_variant<2, uint8_t, false>(r, args, blocks);
        case 3: return dense_variant<3, uint8_t, false>(r, args, blocks);
        default: return dense_variant<4, uint8_t, false>(r, args, blocks);
    }
}

template <int K, int D>
hipError_t bounded_depth_variant(Runner& r, const std::vector<BoundedArgs>& args,
                                 const std::vector<uint32_t>& blocks, bool buf) {
    if (buf)
        return launch(r, kStSgmFinal, sgm_bounded_paths_kernel<Single<BoundedArgs>, K, D, true>,
                      sgm_bounded_paths_kernel<Group<BoundedArgs>, K, D, true>, args, blocks,
                      64 * kWavesPerBlock);
    return launch(r, kStSgmFinal, sgm_bounded_paths_kernel<Single<BoundedArgs>, K, D, false>,
                  sgm_bounded_paths_kernel<Group<BoundedArgs>, K, D, false>, args, blocks,
                  64 * kWavesPerBlock);
}

template <int K>
hipError_t bounded_variant(Runner& r, const std::vector<BoundedArgs>& args,
                           const std::vector<uint32_t>& blocks) {
    // 32-bit buffer offsets when every volume of the launch is below 2^31 bytes
    bool buf = r.tune.bounded_offsets == 32;
    for (const BoundedArgs& a : args)
        buf = buf && (a.dir_stride + a.N) * 2 <= (size_t)INT32_MAX &&
              (size_t)a.H * a.W * sizeof(PixMeta) <= (size_t)INT32_MAX;
    const int d = r.tune.bounded_depth;
    if (d == 4) return bounded_depth_variant<K, 4>(r, args, blocks, buf);
    if (d == 8) return bounded_depth_variant<K, 8>(r, args, blocks, buf);
    return bounded_depth_variant<K, 16>(r, args, blocks, buf);
}

template <int G, int KC>
hipError_t bounded_group_variant(Runner& r, const std::vector<BoundedArgs>& args) {
    std::vector<uint32_t> blocks;
    for (const BoundedArgs& a : args)
        blocks.push_back(div_up(a.lines.base[a.lines.npaths], kB16Waves * (64 / G)));
    return launch(r, kStSgmFinal, sgm_bounded_group_kernel<Single<BoundedArgs>, G, KC>,
                  sgm_bounded_group_kernel<Group<BoundedArgs>, G, KC>, args, blocks,
                  64 * kB16Waves);
}

// Chunks per line (hypotheses / G) rounded up to the compiled variants.
int bounded_chunks(int N, int G) {
    const int c = (N + G - 1) / G;
    if (G == 16) {
        for (int v : {2, 4, 7, 10, 13}) if (c <= v) return v;
        return 16;
    }
    for (int v : {1, 2, 4, 6}) if (c <= v) return v;
    return 8;
}

hipError_t bounded_group(Runner& r, int G, int KC, const std::vector<BoundedArgs>& args) {
    if (G == 16) {
        switch (KC) {
            case 2: return bounded_group_variant<16, 2>(r, args);
            case 4: return bounded_group_variant<16, 4>(r, args);
            case 7: return bounded_group_variant<16, 7>(r, args);
            case 10: return bounded_group_variant<16, 10>(r, args);
            case 13: return bounded_group_variant<16, 13>(r, args);
            default: return bounded_group_variant<16, 16>(r, args);
        }
    }
    switch (KC) {
        case 1: return bounded_group_variant<32, 1>(r, args);
        case 2: return bounded_group_variant<32, 2>(r, args);
        case 4: return bounded_group_variant<32, 4>(r, args);
        case 6: return bounded_group_variant<32, 6>(r, args);
        default: return bounded_group_variant<32, 8>(r, args);
    }
}

hipError_t bounded_k(Runner& r, int K, const std::vector<BoundedArgs>& args,
                     const std::vector<uint32_t>& blocks) {
    switch (K) {
        case 1: return bounded_variant<1>(r, args, blocks);
        case 2: return bounded_variant<2>(r, args, blocks);
        case 3: return bounded_variant<3>(r, args, blocks);
        default: return bounded_variant<4>(r, args, blocks);
    }
}


}  // namespace

int dense_np(int N) { return (N + 3) / 4 * 4; }

// Row stride (elements) of the initial path costs: rows longer than 64 bytes
// take whole 128-byte cache lines, so that the path kernel's non-temporal
// copy-out writes full lines; shorter ones stay packed (4-byte multiples).
int dense_lnp(int N, int elem_bytes) {
    const int rb = dense_np(N) * elem_bytes;
    return rb <= 64 ? dense_np(N) : (rb + 127) / 128 * 128 / elem_bytes;
}

// Row stride of the initial Census cost volume: room for two bytes of 255 after
// the N costs (hypotheses past N read them), within the 256-byte LDS tile rows.
int dense_cvol_np(int N) { return min(dense_np(N + 2), LF_MAX_HYPOTHESES); }

size_t sgm_dense_scratch_bytes(int nv, int H, int W, int N, int npaths, int bits, int P2) {
    const size_t lt = bits + P2 <= 255 ? 1 : 2;
    const size_t cv = round256((size_t)nv * H * W * dense_cvol_np(N));
    // + 256: the row-wise sum reads up to 128 bytes past the last pixel's row
    return cv + (size_t)npaths * nv * H * W * dense_lnp(N, (int)lt) * lt + 256;
}

size_t sgm_bounded_scratch_bytes(int H, int W, int N, int npaths) {
    const size_t meta = round256((size_t)H * W * sizeof(PixMeta));
    return meta + (size_t)npaths * H * W * N * sizeof(uint16_t);
}

hipError_t stage_sgm_initial(Runner& r, const Jobs& jobs, int part) {
    std::vector<CcvArgs> ccv;
    std::vector<uint32_t> ccv_blocks;
    // variants: K in 1..4 x (8-bit, 16-bit, 8-bit with padded rows)
    std::vector<DenseArgs> dense[4][3];
    std::vector<uint32_t> dense_blocks[4][3];
    std::vector<SumWtaArgs> sums[2][2];            // [8/16-bit path costs][8/16 paths]
    std::vector<uint32_t> sum_blocks[2][2];
    std::vector<SumWtaArgs> rows[2];               // 8-bit rows <= 128 B: [8/16 paths]
    std::vector<uint32_t> row_blocks[2];
    std::vector<ExportArgs> ex_cost, ex_sum;       // outputs for checking
    std::vector<uint32_t> ex_cost_blocks, ex_sum_blocks;
    for (const Job* j : jobs) {
        const int H = j->H, W = j->W, N = j->N, NPc = dense_cvol_np(N);
        const size_t HW = (size_t)H * W;
        const lf_sgm_params& sp = j->prm.sgm_init;
        const int bits = j->C * census_bits(j->prm.census);
        const int lt = bits + sp.P2 <= 255 ? 0 : 1;
        const int NP = dense_lnp(N, 1 << lt);
        uint8_t* cvol = (uint8_t*)j->paths;
        void* Lbuf = (char*)j->paths + round256((size_t)j->nv * HW * NPc);
        const int sh = (j->S - 1) / 2, th = (j->T - 1) / 2;

        CcvArgs c{};
        c.cref = j->census;
        c.cview = j->census + (size_t)j->C * HW;
        c.hyp = j->hyp;
        for (int i = 0; i < j->nv; ++i) {
            c.cs4 |= (uint64_t)(uint16_t)(int16_t)(sh - j->st[2 * i]) << (16 * i);
            c.ct4 |= (uint64_t)(uint16_t)(int16_t)(th - j->st[2 * i + 1]) << (16 * i);
        }
        c.nv = j->nv;
        c.C = j->C;
        c.H = H;
        c.W = W;
        c.N = N;
        c.NP = NPc;
        c.tiles = div_up(HW, kTilePix);
        c.cvol = cvol;
        ccv.push_back(c);
        ccv_blocks.push_back(c.tiles * j->nv);

        DenseArgs d{};
        d.cvol = cvol;
        d.Lbuf = Lbuf;
        d.lines = make_lines(H, W, sp.npaths);
        d.nv = j->nv;
        d.H = H;
        d.W = W;
        d.N = N;
        d.NP = NP;
        d.NPc = NPc;
        d.P1 = (uint32_t)sp.P1;
        d.P2 = (uint32_t)sp.P2;
        d.units = make_units(d.lines, H, W);
        d.wblocks = div_up(d.units.nunits, kWavesPerBlock);
        const int K = (N + 63) / 64 - 1;
        const int v = lt == 0 && K <= 1 && bits + 2 * sp.P2 <= 255 + sp.P1 ? 2 : lt;
        dense[K][v].push_back(d);
        dense_blocks[K][v].push_back(d.wblocks * j->nv);

        SumWtaArgs s{};
        s.Lbuf = Lbuf;
        s.HW = (int64_t)HW;
        s.nv = j->nv;
        s.N = N;
        s.NP = NP;
        s.dmap = j->maps;
        const uint32_t ex_blocks = div_up((uint64_t)j->nv * HW * N, 256);
        if (j->ccv_out) {
            ex_cost.push_back(ExportArgs{cvol, j->ccv_out, (int64_t)(j->nv * HW), N, NPc,
                                         sp.npaths, 1});
            ex_cost_blocks.push_back(ex_blocks);
        }
        if (j->csum_init_out) {
            ex_sum.push_back(ExportArgs{Lbuf, j->csum_init_out, (int64_t)(j->nv * HW), N, NP,
                                        sp.npaths, 1 << lt});
            ex_sum_blocks.push_back(ex_blocks);
        }
        const int np16 = sp.npaths == 16 ? 1 : 0;
        if (lt == 0 && NP <= 128) {
            rows[np16].push_back(s);
            row_blocks[np16].push_back(div_up((uint64_t)j->nv * HW, 16));
        } else {
            sums[lt][np16].push_back(s);
            sum_blocks[lt][np16].push_back(div_up((uint64_t)j->nv * HW, 4));
        }
    }
    hipError_t e = hipSuccess;
    using EA = ExportArgs;
    if (part == 0) {
        e = launch(r, kStInitCost, census_cost_volume_kernel<Single<CcvArgs>>,
                   census_cost_volume_kernel<Group<CcvArgs>>, ccv, ccv_blocks, 256);
        if (e == hipSuccess && !ex_cost.empty())
            e = launch(r, kStInitCost, initial_export_kernel<Single<EA>, false>,
                       initial_export_kernel<Group<EA>, false>, ex_cost, ex_cost_blocks, 256);
        return e;
    }
    if (part == 2 && !ex_sum.empty() &&
        (e = launch(r, kStInitSum, initial_export_kernel<Single<EA>, true>,
                    initial_export_kernel<Group<EA>, true>, ex_sum, ex_sum_blocks, 256)) !=
            hipSuccess)
        return e;
    if (part == 1) {
        for (int K = 0; K < 4; ++K)
            for (int v = 0; v < 3; ++v) {
                if (dense[K][v].empty()) continue;
                if ((e = dense_k(r, K + 1, v, dense[K][v], dense_blocks[K][v])) != hipSuccess)
                    return e;
            }
        return hipSuccess;
    }
    // the row-wise sums: one workgroup per 16 pixels (measured faster than
    // persistent workgroups); the others: persistent, each workgroup walks pixels
    constexpr uint32_t kSumGrid = 8192;
    using SA = SumWtaArgs;
    if (!rows[0].empty() &&
        (e = launch(r, kStInitSum, dense_sum_wta_rows_kernel<Single<SA>, 8>,
                    dense_sum_wta_rows_kernel<Group<SA>, 8>, rows[0], row_blocks[0], 256)) !=
            hipSuccess)
        return e;
    if (!rows[1].empty() &&
        (e = launch(r, kStInitSum, dense_sum_wta_rows_kernel<Single<SA>, 16>,
                    dense_sum_wta_rows_kernel<Group<SA>, 16>, rows[1], row_blocks[1], 256)) !=
            hipSuccess)
        return e;
    if (!sums[0][0].empty() &&
        (e = launch(r, kStInitSum, dense_sum_wta_kernel<Single<SA>, uint8_t, 8>,
                    dense_sum_wta_kernel<Group<SA>, uint8_t, 8>, sums[0][0], sum_blocks[0][0],
                    256, kSumGrid)) != hipSuccess)
        return e;
    if (!sums[1][0].empty() &&
        (e = launch(r, kStInitSum, dense_sum_wta_kernel<Single<SA>, uint16_t, 8>,
                    dense_sum_wta_kernel<Group<SA>, uint16_t, 8>, sums[1][0], sum_blocks[1][0],
                    256, kSumGrid)) != hipSuccess)
        return e;
    if (!sums[0][1].empty() &&
        (e = launch(r, kStInitSum, dense_sum_wta_kernel<Single<SA>, uint8_t, 16>,
                    dense_sum_wta_kernel<Group<SA>, uint8_t, 16>, sums[0][1], sum_blocks[0][1],
                    256, kSumGrid)) != hipSuccess)
        return e;
    if (!sums[1][1].empty() &&
        (e = launch(r, kStInitSum, dense_sum_wta_kernel<Single<SA>, uint16_t, 16>,
                    dense_sum_wta_kernel<Group<SA>, uint16_t, 16>, sums[1][1], sum_blocks[1][1],
                    256, kSumGrid)) != hipSuccess)
        return e;
    return hipSuccess;
}

hipError_t stage_sgm_final(Runner& r, const Jobs& jobs) {
    std::vector<MetaArgs> meta;
    std::vector<uint32_t> meta_blocks;
    std::vector<BoundedArgs> paths[4];
    std::vector<uint32_t> path_blocks[4];
    // G lanes per line: [chunks per line] of the compiled variants (at most 16)
    const int G = r.tune.bounded_lanes;
    std::vector<BoundedArgs> grouped[17];
    std::vector<BsumArgs> sums[2][2];              // [16/32-bit sums][8/16 paths]
    std::vector<uint32_t> sum_blocks[2][2];
    for (const Job* j : jobs) {
        const int H = j->H, W = j->W, N = j->N;
        const size_t HW = (size_t)H * W;
        const lf_sgm_params& sp = j->prm.sgm_final;
        PixMeta* pm = (PixMeta*)j->sgm_ws;
        uint16_t* Lbuf = (uint16_t*)((char*)j->sgm_ws + round256(HW * sizeof(PixMeta)));
        const size_t dir_stride = HW * N;          // worst-case cells per direction

        meta.push_back(MetaArgs{j->offsets, j->lo, j->hi, pm, (int)HW, N});
        meta_blocks.push_back(div_up(HW, 256));

        BoundedArgs b{};
        b.cost = j->cost;
        b.meta = pm;
        b.Lbuf = Lbuf;
        b.dir_stride = dir_stride;
        b.lines = make_lines(H, W, sp.npaths);
        b.units = make_units(b.lines, H, W);
        b.H = H;
        b.W = W;
        b.N = N;
        b.P1 = (uint32_t)sp.P1;
        b.P2 = (uint32_t)sp.P2;
        if (G == 16 || G == 32) {
            grouped[bounded_chunks(N, G)].push_back(b);
        } else {
            const int K = (N + 63) / 64 - 1;
            paths[K].push_back(b);
            path_blocks[K].push_back(div_up(b.units.nunits, kWavesPerBlock));
        }

        BsumArgs s{};
        s.Lbuf = Lbuf;
        s.dir_stride = dir_stride;
        s.total = j->offsets + HW;
        s.csum = j->csum;
        s.nblk = std::min<uint32_t>(2048, std::max<uint32_t>(1, div_up(dir_stride, 4096)));
        const int sb = j->prm.sum_bits == 16 ? 0 : 1;
        const int np16 = sp.npaths == 16 ? 1 : 0;
        sums[sb][np16].push_back(s);
        sum_blocks[sb][np16].push_back(s.nblk);
    }
    hipError_t e = launch(r, kStSgmFinal, pix_meta_kernel<Single<MetaArgs>>,
                          pix_meta_kernel<Group<MetaArgs>>, meta, meta_blocks, 256);
    if (e != hipSuccess) return e;
    for (int K = 0; K < 4; ++K) {
        if (paths[K].empty()) continue;
        e = bounded_k(r, K + 1, paths[K], path_blocks[K]);
        if (e != hipSuccess) return e;
    }
    for (int c = 1; c <= 16; ++c) {
        if (grouped[c].empty()) continue;
        if ((e = bounded_group(r, G, c, grouped[c])) != hipSuccess) return e;
    }
    using BA = BsumArgs;
    if (!sums[0][0].empty() &&
        (e = launch(r, kStSgmFinal, bounded_sum_kernel<Single<BA>, uint16_t, 8>,
                    bounded_sum_kernel<Group<BA>, uint16_t, 8>, sums[0][0], sum_blocks[0][0],
                    256)) != hipSuccess)
        return e;
    if (!sums[1][0].empty() &&
        (e = launch(r, kStSgmFinal, bounded_sum_kernel<Single<BA>, uint32_t, 8>,
                    bounded_sum_kernel<Group<BA>, uint32_t, 8>, sums[1][0], sum_blocks[1][0],
                    256)) != hipSuccess)
        return e;
    if (!sums[0][1].empty() &&
        (e = launch(r, kStSgmFinal, bounded_sum_kernel<Single<BA>, uint16_t, 16>,
                    bounded_sum_kernel<Group<BA>, uint16_t, 16>, sums[0][1], sum_blocks[0][1],
                    256)) != hipSuccess)
        return e;
    if (!sums[1][1].empty() &&
        (e = launch(r, kStSgmFinal, bounded_sum_kernel<Single<BA>, uint32_t, 16>,
                    bounded_sum_kernel<Group<BA>, uint32_t, 16>, sums[1][1], sum_blocks[1][1],
                    256)) != hipSuccess)
        return e;
    return hipSuccess;
}

}  // namespace lf
