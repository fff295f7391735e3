// Internal declarations of liblf: device helpers and the host-side launchers each
// kernel file provides to the API layer (api.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/lf.h"

namespace lf {

constexpr uint32_t kInf = 0x3FFFFFFFu;   // +inf of the SGM path recurrences
constexpr int kMaxCensusRadius = 7;      // windows up to 15 x 15
constexpr int kMaxBatchImages = 8;

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return min(max(x, lo), hi); }

// Loads one view sample as float (8-bit values convert exactly).
template <typename T> __device__ __forceinline__ float ld(const T* p) { return (float)*p; }

// Census of up to kMaxBatchImages images sharing a size; image z starts at
// base + off[z] elements.  When n > kMaxBatchImages the images are taken at a
// constant stride: off[z] = z * stride.
struct CensusBatch {
    const void* base;
    int64_t off[kMaxBatchImages];
    int64_t stride;
    int n;
};

hipError_t launch_census(const CensusBatch& b, int dtype, int H, int W, int pitch, int win_h,
                         int win_w, uint64_t* out, hipStream_t st);

// --- SGM -------------------------------------------------------------------
struct SgmDense {                // initial stage: Census cost on the fly, all N hypotheses
    const uint64_t* cref;        // [H*W]
    const uint64_t* cview;       // [nv][H*W]
    int16_t* dmap;               // [nv][H*W] WTA result
    int cs[4], ct[4];            // s_hat - s, t_hat - t of each cross view
    int nv;
};

struct SgmBounded {              // final stage: CSR volume over per-pixel ranges
    const uint16_t* cost;
    const int64_t* off;          // [H*W+1]; off[H*W] is the cell count
    const int16_t* lo;
    const int16_t* hi;
    void* csum;                  // uint16 or uint32 [cells]
    int sum_bits;
};

// Scratch for the per-direction path costs (bytes).
size_t sgm_dense_scratch_bytes(int nv, int H, int W, int N, int npaths, int bits, int P2);
size_t sgm_bounded_scratch_bytes(int H, int W, int N, int npaths);

// bits: Census string length (bounds the initial cost); scratch: see above.
hipError_t launch_sgm_dense(const SgmDense& a, const float* hyp, int H, int W, int N, int P1,
                            int P2, int npaths, int bits, void* scratch, hipStream_t st);
hipError_t launch_sgm_bounded(const SgmBounded& a, int H, int W, int N, int P1, int P2,
                              int npaths, void* scratch, hipStream_t st);

// --- per-pixel stages ------------------------------------------------------
hipError_t launch_fuse(const int16_t* maps, int nv, int HW, int phi, int16_t* dinit,
                       hipStream_t st);
hipError_t launch_fill(const int16_t* in, int16_t* out, int H, int W, hipStream_t st);
hipError_t launch_borders(const int16_t* dinit, const void* ref, int dtype, int pitch, int H,
                          int W, int N, int lambda, float alpha, float tau, int16_t* lo,
                          int16_t* hi, hipStream_t st);

// exclusive prefix sum of range widths -> offsets[HW+1]; scratch >= scan_scratch_bytes(HW)
size_t scan_scratch_bytes(int64_t HW);
hipError_t launch_offsets(const int16_t* lo, const int16_t* hi, int64_t HW, int64_t* offsets,
                          void* scratch, hipStream_t st);

hipError_t launch_cost_l2(const void* views, int dtype, int S, int T, int H, int W, int pitch,
                          const float* hyp, int N, const int16_t* lo, const int16_t* hi,
                          const int64_t* off, float alpha, int32_t cap, uint16_t* cost,
                          float* cost_f32, int64_t cap_cells, hipStream_t st);
hipError_t launch_cost_census_all(const uint64_t* census_all, int S, int T, int H, int W,
                                  const float* hyp, int N, const int16_t* lo, const int16_t* hi,
                                  const int64_t* off, int32_t cap, uint16_t* cost,
                                  float* cost_f32, int64_t cap_cells, hipStream_t st);

hipError_t launch_wta_subpixel(const void* csum, int sum_bits, const int64_t* off,
                               const int16_t* lo, const int16_t* hi, int H, int W,
                               const float* hyp, int16_t* d_index, float* disp,
                               hipStream_t st);
hipError_t launch_median3(const float* in, float* out, int H, int W, hipStream_t st);

}  // namespace lf
