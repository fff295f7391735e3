/*
 * lfo.h -- plain single-threaded CPU oracle for the light-field depth method of
 * "Rapid Light Field Depth Estimation with Semi-Global Matching" (Anisimov,
 * Wasenmueller, Stricker, 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; it is
 * loaded by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark, and by nothing else.  It shares no code, header, table or helper
 * with the GPU library: its own types, its own loops, written for a reader who
 * checks it against the paper by eye.
 *
 * Conventions (all arrays host memory, row-major, caller-allocated):
 *   views   float32 [T][S][H][W]; 8-bit inputs are passed converted (exactly).
 *   hyp     float32 [N], the disparity hypotheses d_0 < ... < d_{N-1}.
 *   volumes "dense frame" [H][W][N]: entry (v, u, k) at ((v*W)+u)*N + k; entries
 *           whose k lies outside a pixel's range [lo, hi] are left untouched.
 *   lo/hi   int16 [H][W] per-pixel index range, or NULL for the full range.
 *   s_hat = (S-1)/2, t_hat = (T-1)/2 (S and T odd): the reference view.
 *
 * Every function states the passage of the paper it follows.  Readings of the
 * paper where it is silent or garbled are stated where they are used.
 */
#ifndef LFO_H
#define LFO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Census transform, Sec. 3.2 Eq. (2)-(3): bit n (LSB first) compares the centre
 * with the n-th window neighbour in row-major order, centre skipped; the bit is 1
 * iff centre > neighbour.  Neighbours outside the image are clamped to the edge.
 * Window: win_h rows x win_w cols, both odd, win_h*win_w - 1 <= 64. */
void lfo_census(const float* img, int H, int W, int win_h, int win_w, uint64_t* out);

/* Census transform over a caller-given neighbour set (Sec. 3.2: a sparse window
 * compares the centre with only some of the window's pixels): bit n (LSB first)
 * compares the centre with the pixel at row offset dy[n], column offset dx[n]; 1
 * iff centre > neighbour; clamped to the edge.  0 <= n_off <= 64.  The dense
 * window is the special case of every offset of the window in row-major order,
 * the centre skipped. */
void lfo_census_offsets(const float* img, int H, int W, int n_off, const int* dy,
                        const int* dx, uint64_t* out);

/* Hamming distance, Eq. (5). */
int lfo_hamming(uint64_t a, uint64_t b);

/* Cross-lying view set V of Sec. 3.4: (s_hat,0), (s_hat,T-1), (0,t_hat),
 * (S-1,t_hat), dropping entries equal to the reference view and duplicates.
 * Writes (s,t) pairs to out[2*i], out[2*i+1]; returns |V|. */
int lfo_cross_views(int S, int T, int* out);

/* Initial Census cost for one cross view, Eq. (7): C(p,k) = HD(Lc_ref(p),
 * Lc_view(p + shift)), the shift rounded to the nearest pixel, Eq. (1):
 * du = rint(cs*d_k), dv = rint(ct*d_k) with cs = s_hat - s, ct = t_hat - t,
 * products and rounding in float32 (half to even).  Sampled position clamped. */
void lfo_cost_census_view(const uint64_t* cref, const uint64_t* cview, int H, int W,
                          int cs, int ct, const float* hyp, int N, int32_t* cost);

/* One SGM path direction r = (du, dv), Eq. (8).  With literal = 0 the recurrence
 * subtracts m = min_j L_r(p-r, j) (the normalised form; it differs from Eq. (8)
 * by a per-pixel constant); with literal = 1 it is Eq. (8) as printed.  Terms
 * whose index lies outside the range of p-r are omitted.  The first pixel of a
 * path (p-r outside the image) takes L_r = C.  L is [H][W][N] int64. */
void lfo_sgm_path(const int32_t* cost, const int16_t* lo, const int16_t* hi,
                  int H, int W, int N, int du, int dv, int P1, int P2, int literal,
                  int64_t* L);

/* Sum over path directions, Eq. (9), normalised form.  npaths = 8: the four axis
 * and four diagonal directions; npaths = 16 adds (+-1,+-2) and (+-2,+-1). */
void lfo_sgm(const int32_t* cost, const int16_t* lo, const int16_t* hi, int H, int W,
             int N, int P1, int P2, int npaths, int64_t* csum);

/* Winner-take-all, Eq. (10): lowest index k in [lo, hi] with minimal csum. */
void lfo_wta(const int64_t* csum, const int16_t* lo, const int16_t* hi, int H, int W,
             int N, int16_t* idx);

/* Fusion of the intermediate maps D_1..D_nv with confidence threshold phi
 * (Sec. 3.4): D_init = D_1; for i >= 2, if the pixel is still valid and
 * |D_init - D_i| < phi, D_init becomes the (floored) average of the two,
 * otherwise the pixel is invalid (-1) for good. maps: [nv][H][W]. */
void lfo_fuse(const int16_t* maps, int nv, int H, int W, int phi, int16_t* dinit);

/* One median hole-filling pass (Sec. 3.4, window 3 per Sec. 4.3): an invalid
 * pixel takes the lower median of the valid pixels among its 8 neighbours
 * inside the image; valid pixels are copied; reads `in` only (Jacobi). */
void lfo_fill(const int16_t* in, int H, int W, int16_t* out);

/* Sobel edge mask on the reference view (Sec. 3.4): G = |Gx| + |Gy| of the 3x3
 * Sobel operator, clamp-to-edge, float32; edge iff alpha*G > tau.  ref: C planes;
 * colour takes the largest G over the channels. */
void lfo_edges(const float* ref, int C, int H, int W, float alpha, float tau, uint8_t* edge);

/* Borders, Eq. (11): valid, non-edge pixel: lo = max(0, D_init - lambda),
 * hi = min(N-1, D_init + lambda); invalid or edge pixel: the full range.
 * lambda < 0 selects the boundary-less search (Sec. 4.5): the full range for
 * every pixel (the initial map is then unused). */
void lfo_borders(const int16_t* dinit, const uint8_t* edge, int H, int W, int N,
                 int lambda, int lambda_far, int16_t* lo, int16_t* hi);

/* Border half-width at initial index d (Sec. 4.6, adaptive by depth): lambda_far
 * at k = 0 (the smallest disparity, the farthest point) falling linearly to
 * lambda at k = N-1, rounded half up; lambda_far <= lambda keeps lambda. */
int lfo_border_width(int lambda, int lambda_far, int d, int N);

/* Bounded l2 matching cost over all views, Eq. (12), in double precision:
 * S(p,k) = sum_t sum_s |L_ref(p) - B_{s,t}(u + cs*d_k, v + ct*d_k)| with B the
 * bilinear interpolation of view (s,t), taps clamped to the image.  views:
 * [T][S][C][H][W]; with C > 1 channels the term is the l2 norm of the colour
 * difference, sqrt(sum_c (ref_c - B_c)^2). */
void lfo_cost_l2_f64(const float* views, int S, int T, int C, int H, int W, const float* hyp,
                     int N, const int16_t* lo, const int16_t* hi, double* out);

/* The same sum in float32, in the order t outer, s inner, starting from +0:
 * shift sh = (float)cs * d_k rounded once, x0 = floor(sh), fx = sh - x0 (exact);
 * top = fma(fx, b-a, a), bot = fma(fx, e-c, c), val = fma(fy, bot-top, top);
 * acc += |ref - val| (C = 1) or, with dl_c = ref_c - val_c,
 * acc += sqrtf(fma(dl_2, dl_2, fma(dl_1, dl_1, dl_0 * dl_0))) (C = 3).  This is the
 * precision the quantised cost is decided in. */
void lfo_cost_l2_f32(const float* views, int S, int T, int C, int H, int W, const float* hyp,
                     int N, const int16_t* lo, const int16_t* hi, float* out);

/* Quantisation to the integer SGM domain: C = min(rint(alpha*S), cap), with the
 * product and rounding in float32. */
void lfo_quantize(const float* s, int H, int W, int N, const int16_t* lo,
                  const int16_t* hi, float alpha, int32_t cap, int32_t* cost);

/* Census cost over all views, Eq. (15): S(p,k) = sum_t sum_s HD(Lc_ref(p),
 * Lc_{s,t}(p + rounded shift)), then C = min(S, cap).  census_all: [T][S][C][H][W];
 * colour: the Hamming distances of the C channels are summed. */
void lfo_cost_census_all(const uint64_t* census_all, int S, int T, int C, int H, int W,
                         const float* hyp, int N, const int16_t* lo, const int16_t* hi,
                         int32_t cap, int32_t* cost);

/* Sub-pixel refinement, Sec. 3.6 Eq. (13) with the parabola vertex
 * o = (c- - c+) / (2 (c- + c+ - 2 c0)), applied when k*-1 >= lo, k*+1 <= hi and
 * hi - lo >= 4; otherwise o = 0.  Output disparity (float32):
 * o >= 0: fma(o, d[k*+1]-d[k*], d[k*]); o < 0: fma(o, d[k*]-d[k*-1], d[k*]). */
void lfo_subpixel(const int64_t* csum, const int16_t* lo, const int16_t* hi,
                  const int16_t* idx, const float* hyp, int H, int W, int N, float* disp);

/* 3x3 median filter (Sec. 3.6), clamp-to-edge. */
void lfo_median3(const float* in, int H, int W, float* out);

/* Quantisation cap of the final cost: cap + 2*P2 <= 65535 keeps 16-bit path
 * costs exact next to a +inf sentinel of 65535; with 16-bit sums it also keeps
 * npaths*(cap + P2) <= 65535. */
int32_t lfo_cost_cap(int P2_final, int npaths, int sum_bits);

/* Whole-method parameters (own definition; not shared with the GPU library). */
typedef struct {
    int win_h, win_w;         /* Census window */
    int P1_init, P2_init;     /* SGM penalties, initial stage */
    int P1_final, P2_final;   /* SGM penalties, final stage */
    int npaths;               /* 8 or 16 */
    int phi, lambda, fill_passes;
    int lambda_far;           /* adaptive border (Sec. 4.6); <= lambda: off */
    int channels;             /* planes per view: 1 (grayscale) or 3 (colour) */
    float edge_tau;           /* +inf disables the edge exclusion */
    float alpha;              /* cost scale to 8-bit units */
    int cost_kind;            /* 0 = l2 (Eq. 12), 1 = Census (Eq. 15) */
    int median;               /* 0 = off, 3 = 3x3 */
    int32_t cost_cap;         /* quantisation cap of the final cost */
    int n_offsets;            /* 0: the dense win_h x win_w window; 1..64: the sparse
                                 neighbour set off_dy/off_dx (lfo_census_offsets) */
    int off_dy[64], off_dx[64];
} lfo_params;

/* The whole method, Sec. 3.3-3.6.  Optional outputs may be NULL:
 * maps [|V|][H][W], dinit/lo/hi [H][W], cost/csum dense [H][W][N] (final stage),
 * init_cost [|V|][H][W][N] (Eq. 7, channels summed) and init_csum [|V|][H][W][N]
 * (Eq. 9 over the initial stage's paths) of every cross view.
 * Returns 0, or -1 on invalid arguments. */
int lfo_depth(const float* views, int S, int T, int H, int W, const float* hyp, int N,
              const lfo_params* prm, float* disparity, int16_t* d_index,
              int16_t* maps, int16_t* dinit, int16_t* lo, int16_t* hi,
              int32_t* cost, int64_t* csum, int32_t* init_cost, int64_t* init_csum);

#ifdef __cplusplus
}
#endif
#endif
