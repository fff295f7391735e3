/*
 * lfo.c -- plain single-threaded CPU oracle of the light-field depth method
 * (Anisimov, Wasenmueller, Stricker 2019).  TEST INFRASTRUCTURE ONLY: see lfo.h.
 *
 * Built with -O3 -ffp-contract=off and without -ffast-math, so every float
 * operation is the one written here (fmaf only where written).
 */
#include "lfo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

static int range_lo(const int16_t* lo, size_t p) { return lo ? lo[p] : 0; }
static int range_hi(const int16_t* hi, size_t p, int N) { return hi ? hi[p] : N - 1; }

/* ---------------------------------------------------------------- Census */
/* Sec. 3.2, Eq. (2)-(3). */
void lfo_census(const float* img, int H, int W, int win_h, int win_w, uint64_t* out)
{
    int rh = win_h / 2, rw = win_w / 2;
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            float centre = img[(size_t)v * W + u];
            uint64_t bits = 0;
            int n = 0;
            for (int i = -rh; i <= rh; ++i) {
                for (int j = -rw; j <= rw; ++j) {
                    if (i == 0 && j == 0) continue;          /* the centre is skipped */
                    int y = clampi(v + i, 0, H - 1);
                    int x = clampi(u + j, 0, W - 1);
                    float nb = img[(size_t)y * W + x];
                    if (centre > nb) bits |= (uint64_t)1 << n; /* xi = 1 iff p1 > p2 */
                    ++n;
                }
            }
            out[(size_t)v * W + u] = bits;
        }
    }
}

/* Sec. 3.2, sparse window: the same comparison of Eq. (3), over the listed
 * neighbours only, bit n for the n-th entry of the list. */
void lfo_census_offsets(const float* img, int H, int W, int n_off, const int* dy,
                        const int* dx, uint64_t* out)
{
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            float centre = img[(size_t)v * W + u];
            uint64_t bits = 0;
            for (int n = 0; n < n_off; ++n) {
                int y = clampi(v + dy[n], 0, H - 1);
                int x = clampi(u + dx[n], 0, W - 1);
                if (centre > img[(size_t)y * W + x]) bits |= (uint64_t)1 << n;
            }
            out[(size_t)v * W + u] = bits;
        }
    }
}

/* Census of one plane with the window the parameters name. */
static void census_of(const lfo_params* prm, const float* img, int H, int W, uint64_t* out)
{
    if (prm->n_offsets > 0)
        lfo_census_offsets(img, H, W, prm->n_offsets, prm->off_dy, prm->off_dx, out);
    else
        lfo_census(img, H, W, prm->win_h, prm->win_w, out);
}

/* Eq. (5): number of differing bit positions. */
int lfo_hamming(uint64_t a, uint64_t b)
{
    uint64_t x = a ^ b;
    int n = 0;
    for (int i = 0; i < 64; ++i) n += (int)((x >> i) & 1u);
    return n;
}

/* ---------------------------------------------------------- cross views */
/* Sec. 3.4: V = {(s_hat,0), (s_hat,t_max), (0,t_hat), (s_max,t_hat)}. */
int lfo_cross_views(int S, int T, int* out)
{
    int sh = (S - 1) / 2, th = (T - 1) / 2;
    int cand[4][2] = {{sh, 0}, {sh, T - 1}, {0, th}, {S - 1, th}};
    int n = 0;
    for (int i = 0; i < 4; ++i) {
        int s = cand[i][0], t = cand[i][1];
        if (s == sh && t == th) continue;            /* the reference view itself */
        int dup = 0;
        for (int j = 0; j < n; ++j)
            if (out[2 * j] == s && out[2 * j + 1] == t) dup = 1;
        if (dup) continue;
        out[2 * n] = s;
        out[2 * n + 1] = t;
        ++n;
    }
    return n;
}

/* ------------------------------------------------------- initial cost */
/* Eq. (7) with the matching position of Eq. (1), rounded to the nearest pixel. */
void lfo_cost_census_view(const uint64_t* cref, const uint64_t* cview, int H, int W,
                          int cs, int ct, const float* hyp, int N, int32_t* cost)
{
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            for (int k = 0; k < N; ++k) {
                float shu = (float)cs * hyp[k];
                float shv = (float)ct * hyp[k];
                int x = clampi(u + (int)rintf(shu), 0, W - 1);
                int y = clampi(v + (int)rintf(shv), 0, H - 1);
                cost[p * N + k] = lfo_hamming(cref[p], cview[(size_t)y * W + x]);
            }
        }
    }
}

/* ----------------------------------------------------------------- SGM */
/* Eq. (8), one direction; see lfo.h for the normalised form and ranges. */
void lfo_sgm_path(const int32_t* cost, const int16_t* lo, const int16_t* hi,
                  int H, int W, int N, int du, int dv, int P1, int P2, int literal,
                  int64_t* L)
{
    for (int vi = 0; vi < H; ++vi) {
        int v = dv >= 0 ? vi : H - 1 - vi;
        for (int ui = 0; ui < W; ++ui) {
            int u = du >= 0 ? ui : W - 1 - ui;
            size_t p = (size_t)v * W + u;
            int plo = range_lo(lo, p), phi = range_hi(hi, p, N);
            int qu = u - du, qv = v - dv;
            if (qu < 0 || qu >= W || qv < 0 || qv >= H) {
                /* first pixel of the path */
                for (int k = plo; k <= phi; ++k) L[p * N + k] = cost[p * N + k];
                continue;
            }
            size_t q = (size_t)qv * W + qu;
            int qlo = range_lo(lo, q), qhi = range_hi(hi, q, N);
            int64_t m = INT64_MAX;
            for (int j = qlo; j <= qhi; ++j)
                if (L[q * N + j] < m) m = L[q * N + j];
            for (int k = plo; k <= phi; ++k) {
                int64_t best = m + P2;
                if (k >= qlo && k <= qhi && L[q * N + k] < best) best = L[q * N + k];
                if (k - 1 >= qlo && k - 1 <= qhi && L[q * N + k - 1] + P1 < best)
                    best = L[q * N + k - 1] + P1;
                if (k + 1 >= qlo && k + 1 <= qhi && L[q * N + k + 1] + P1 < best)
                    best = L[q * N + k + 1] + P1;
                L[p * N + k] = cost[p * N + k] + best - (literal ? 0 : m);
            }
        }
    }
}

static const int DIRS16[16][2] = {
    {1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}, {1, -1}, {-1, 1},
    {1, 2}, {-1, -2}, {2, 1}, {-2, -1}, {2, -1}, {-2, 1}, {1, -2}, {-1, 2}};

/* Eq. (9). */
void lfo_sgm(const int32_t* cost, const int16_t* lo, const int16_t* hi, int H, int W,
             int N, int P1, int P2, int npaths, int64_t* csum)
{
    size_t n = (size_t)H * W * N;
    int64_t* L = (int64_t*)malloc(n * sizeof(int64_t));
    memset(csum, 0, n * sizeof(int64_t));
    for (int r = 0; r < npaths; ++r) {
        lfo_sgm_path(cost, lo, hi, H, W, N, DIRS16[r][0], DIRS16[r][1], P1, P2, 0, L);
        for (size_t p = 0; p < (size_t)H * W; ++p) {
            int plo = range_lo(lo, p), phi = range_hi(hi, p, N);
            for (int k = plo; k <= phi; ++k) csum[p * N + k] += L[p * N + k];
        }
    }
    free(L);
}

/* Eq. (10); ties resolve to the lowest index. */
void lfo_wta(const int64_t* csum, const int16_t* lo, const int16_t* hi, int H, int W,
             int N, int16_t* idx)
{
    for (size_t p = 0; p < (size_t)H * W; ++p) {
        int plo = range_lo(lo, p), phi = range_hi(hi, p, N);
        int best = plo;
        for (int k = plo + 1; k <= phi; ++k)
            if (csum[p * N + k] < csum[p * N + best]) best = k;
        idx[p] = (int16_t)best;
    }
}

/* ------------------------------------------------- fusion, fill, borders */
void lfo_fuse(const int16_t* maps, int nv, int H, int W, int phi, int16_t* dinit)
{
    size_t np = (size_t)H * W;
    for (size_t p = 0; p < np; ++p) {
        int acc = maps[p];
        int valid = 1;
        for (int i = 1; i < nv; ++i) {
            int di = maps[(size_t)i * np + p];
            if (valid && abs(acc - di) < phi)
                acc = (acc + di) / 2;   /* indices are >= 0: this is the floor */
            else
                valid = 0;
        }
        dinit[p] = (int16_t)(valid ? acc : -1);
    }
}

void lfo_fill(const int16_t* in, int H, int W, int16_t* out)
{
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            if (in[p] >= 0) { out[p] = in[p]; continue; }
            int vals[8], n = 0;
            for (int i = -1; i <= 1; ++i)
                for (int j = -1; j <= 1; ++j) {
                    if (i == 0 && j == 0) continue;
                    int y = v + i, x = u + j;
                    if (y < 0 || y >= H || x < 0 || x >= W) continue;
                    int d = in[(size_t)y * W + x];
                    if (d >= 0) vals[n++] = d;
                }
            if (n == 0) { out[p] = -1; continue; }
            /* insertion sort, then the lower median */
            for (int a = 1; a < n; ++a) {
                int key = vals[a], b = a - 1;
                while (b >= 0 && vals[b] > key) { vals[b + 1] = vals[b]; --b; }
                vals[b + 1] = key;
            }
            out[p] = (int16_t)vals[(n - 1) / 2];
        }
    }
}

void lfo_edges(const float* ref, int C, int H, int W, float alpha, float tau, uint8_t* edge)
{
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            int ym = clampi(v - 1, 0, H - 1), yp = clampi(v + 1, 0, H - 1);
            int xm = clampi(u - 1, 0, W - 1), xp = clampi(u + 1, 0, W - 1);
            float g = 0.0f;
            for (int c = 0; c < C; ++c) {       /* colour: the strongest channel */
                const float* img = ref + (size_t)c * H * W;
#define I(y, x) img[(size_t)(y) * W + (x)]
                float gx = ((I(ym, xp) + 2.0f * I(v, xp)) + I(yp, xp))
                         - ((I(ym, xm) + 2.0f * I(v, xm)) + I(yp, xm));
                float gy = ((I(yp, xm) + 2.0f * I(yp, u)) + I(yp, xp))
                         - ((I(ym, xm) + 2.0f * I(ym, u)) + I(ym, xp));
#undef I
                float gc = fabsf(gx) + fabsf(gy);
                if (gc > g) g = gc;
            }
            edge[(size_t)v * W + u] = (uint8_t)(alpha * g > tau);
        }
    }
}

int lfo_border_width(int lambda, int lambda_far, int d, int N)
{
    /* Sec. 4.6: a wider border for small disparities (far objects).  Linear in
     * the index from lambda_far at k = 0 to lambda at k = N-1, rounded half up. */
    if (lambda_far <= lambda || N < 2) return lambda;
    return lambda + ((lambda_far - lambda) * (N - 1 - d) + (N - 1) / 2) / (N - 1);
}

void lfo_borders(const int16_t* dinit, const uint8_t* edge, int H, int W, int N,
                 int lambda, int lambda_far, int16_t* lo, int16_t* hi)
{
    for (size_t p = 0; p < (size_t)H * W; ++p) {
        int d = dinit[p];
        /* lambda < 0: the boundary-less search of Sec. 4.5 -- every pixel keeps T */
        if (lambda < 0 || d < 0 || (edge && edge[p])) {
            lo[p] = 0;
            hi[p] = (int16_t)(N - 1);
        } else {
            int lam = lfo_border_width(lambda, lambda_far, d, N);
            lo[p] = (int16_t)(d - lam < 0 ? 0 : d - lam);
            hi[p] = (int16_t)(d + lam > N - 1 ? N - 1 : d + lam);
        }
    }
}

/* ----------------------------------------------------- bounded l2 cost */
void lfo_cost_l2_f64(const float* views, int S, int T, int C, int H, int W, const float* hyp,
                     int N, const int16_t* lo, const int16_t* hi, double* out)
{
    int sh = (S - 1) / 2, th = (T - 1) / 2;
    size_t plane = (size_t)H * W;
    const float* ref = views + ((size_t)th * S + sh) * C * plane;
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            int plo = range_lo(lo, p), phi = range_hi(hi, p, N);
            for (int k = plo; k <= phi; ++k) {
                double acc = 0.0;
                for (int t = 0; t < T; ++t) {
                    for (int s = 0; s < S; ++s) {
                        double x = (double)u + (double)(sh - s) * (double)hyp[k];
                        double y = (double)v + (double)(th - t) * (double)hyp[k];
                        double x0 = floor(x), y0 = floor(y);
                        double fx = x - x0, fy = y - y0;
                        int xa = clampi((int)x0, 0, W - 1), xb = clampi((int)x0 + 1, 0, W - 1);
                        int ya = clampi((int)y0, 0, H - 1), yb = clampi((int)y0 + 1, 0, H - 1);
                        double sq = 0.0, dist = 0.0;
                        for (int ch = 0; ch < C; ++ch) {
                            const float* view = views + (((size_t)t * S + s) * C + ch) * plane;
                            double a = view[(size_t)ya * W + xa], b = view[(size_t)ya * W + xb];
                            double c = view[(size_t)yb * W + xa], e = view[(size_t)yb * W + xb];
                            double top = a + fx * (b - a);
                            double bot = c + fx * (e - c);
                            double val = top + fy * (bot - top);
                            double dl = (double)ref[ch * plane + p] - val;
                            dist = fabs(dl);
                            sq += dl * dl;
                        }
                        /* the l2 norm of the colour difference, R16 */
                        acc += C == 1 ? dist : sqrt(sq);
                    }
                }
                out[p * N + k] = acc;
            }
        }
    }
}

void lfo_cost_l2_f32(const float* views, int S, int T, int C, int H, int W, const float* hyp,
                     int N, const int16_t* lo, const int16_t* hi, float* out)
{
    int sh = (S - 1) / 2, th = (T - 1) / 2;
    size_t plane = (size_t)H * W;
    const float* ref = views + ((size_t)th * S + sh) * C * plane;
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            int plo = range_lo(lo, p), phi = range_hi(hi, p, N);
            for (int k = plo; k <= phi; ++k) {
                float acc = 0.0f;
                for (int t = 0; t < T; ++t) {
                    float shy = (float)(th - t) * hyp[k];
                    float y0 = floorf(shy);
                    float fy = shy - y0;
                    int ya = clampi(v + (int)y0, 0, H - 1), yb = clampi(v + (int)y0 + 1, 0, H - 1);
                    for (int s = 0; s < S; ++s) {
                        float shx = (float)(sh - s) * hyp[k];
                        float x0 = floorf(shx);
                        float fx = shx - x0;
                        int xa = clampi(u + (int)x0, 0, W - 1), xb = clampi(u + (int)x0 + 1, 0, W - 1);
                        float sq = 0.0f, dist = 0.0f;
                        for (int ch = 0; ch < C; ++ch) {
                            const float* view = views + (((size_t)t * S + s) * C + ch) * plane;
                            float a = view[(size_t)ya * W + xa], b = view[(size_t)ya * W + xb];
                            float c = view[(size_t)yb * W + xa], e = view[(size_t)yb * W + xb];
                            float top = fmaf(fx, b - a, a);
                            float bot = fmaf(fx, e - c, c);
                            float val = fmaf(fy, bot - top, top);
                            float dl = ref[ch * plane + p] - val;
                            dist = fabsf(dl);
                            /* channel 0 squared, the others added by fma in order */
                            sq = ch == 0 ? dl * dl : fmaf(dl, dl, sq);
                        }
                        acc = acc + (C == 1 ? dist : sqrtf(sq));
                    }
                }
                out[p * N + k] = acc;
            }
        }
    }
}

void lfo_quantize(const float* s, int H, int W, int N, const int16_t* lo,
                  const int16_t* hi, float alpha, int32_t cap, int32_t* cost)
{
    for (size_t p = 0; p < (size_t)H * W; ++p) {
        int plo = range_lo(lo, p), phi = range_hi(hi, p, N);
        for (int k = plo; k <= phi; ++k) {
            float q = rintf(alpha * s[p * N + k]);
            cost[p * N + k] = q > (float)cap ? cap : (int32_t)q;
        }
    }
}

void lfo_cost_census_all(const uint64_t* census_all, int S, int T, int C, int H, int W,
                         const float* hyp, int N, const int16_t* lo, const int16_t* hi,
                         int32_t cap, int32_t* cost)
{
    int sh = (S - 1) / 2, th = (T - 1) / 2;
    size_t plane = (size_t)H * W;
    const uint64_t* cref = census_all + ((size_t)th * S + sh) * C * plane;
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            int plo = range_lo(lo, p), phi = range_hi(hi, p, N);
            for (int k = plo; k <= phi; ++k) {
                int64_t acc = 0;
                for (int t = 0; t < T; ++t)
                    for (int s = 0; s < S; ++s) {
                        int x = clampi(u + (int)rintf((float)(sh - s) * hyp[k]), 0, W - 1);
                        int y = clampi(v + (int)rintf((float)(th - t) * hyp[k]), 0, H - 1);
                        for (int ch = 0; ch < C; ++ch) {  /* per-channel Census, summed */
                            const uint64_t* cv = census_all + (((size_t)t * S + s) * C + ch) * plane;
                            acc += lfo_hamming(cref[ch * plane + p], cv[(size_t)y * W + x]);
                        }
                    }
                cost[p * N + k] = acc > cap ? cap : (int32_t)acc;
            }
        }
    }
}

/* ------------------------------------------------------ post-processing */
void lfo_subpixel(const int64_t* csum, const int16_t* lo, const int16_t* hi,
                  const int16_t* idx, const float* hyp, int H, int W, int N, float* disp)
{
    for (size_t p = 0; p < (size_t)H * W; ++p) {
        int plo = range_lo(lo, p), phi = range_hi(hi, p, N);
        int k = idx[p];
        if (k - 1 >= plo && k + 1 <= phi && phi - plo >= 4) {
            int64_t cm = csum[p * N + k - 1], c0 = csum[p * N + k], cp = csum[p * N + k + 1];
            float o = (float)(cm - cp) / (2.0f * (float)(cm + cp - 2 * c0));
            if (o >= 0.0f)
                disp[p] = fmaf(o, hyp[k + 1] - hyp[k], hyp[k]);
            else
                disp[p] = fmaf(o, hyp[k] - hyp[k - 1], hyp[k]);
        } else {
            disp[p] = hyp[k];
        }
    }
}

void lfo_median3(const float* in, int H, int W, float* out)
{
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            float w[9];
            int n = 0;
            for (int i = -1; i <= 1; ++i)
                for (int j = -1; j <= 1; ++j)
                    w[n++] = in[(size_t)clampi(v + i, 0, H - 1) * W + clampi(u + j, 0, W - 1)];
            for (int a = 1; a < 9; ++a) {
                float key = w[a];
                int b = a - 1;
                while (b >= 0 && w[b] > key) { w[b + 1] = w[b]; --b; }
                w[b + 1] = key;
            }
            out[(size_t)v * W + u] = w[4];
        }
    }
}

int32_t lfo_cost_cap(int P2_final, int npaths, int sum_bits)
{
    int32_t cap = 65535 - 2 * P2_final;
    if (sum_bits == 16 && 65535 / npaths - P2_final < cap) cap = 65535 / npaths - P2_final;
    return cap;
}

/* ------------------------------------------------------- whole method */
int lfo_depth(const float* views, int S, int T, int H, int W, const float* hyp, int N,
              const lfo_params* prm, float* disparity, int16_t* d_index,
              int16_t* maps_out, int16_t* dinit_out, int16_t* lo_out, int16_t* hi_out,
              int32_t* cost_out, int64_t* csum_out, int32_t* init_cost_out,
              int64_t* init_csum_out)
{
    if (S < 1 || T < 1 || (S % 2) == 0 || (T % 2) == 0 || S * T < 2 || H < 1 || W < 1 || N < 2)
        return -1;
    if (prm->n_offsets < 0 || prm->n_offsets > 64) return -1;
    const int C = prm->channels < 1 ? 1 : prm->channels;
    size_t plane = (size_t)H * W, vol = plane * N;
    int sh = (S - 1) / 2, th = (T - 1) / 2;
    /* views [T][S][C][H][W]: a view is C planes (one for grayscale) */
    const float* ref = views + ((size_t)th * S + sh) * C * plane;

    /* Sec. 3.4: Census cost on the cross-lying views, SGM, WTA -> D_1..D_|V|.
     * Colour views: Census per channel, Hamming distances summed (Sec. 3.2). */
    int vset[8];
    int nv = lfo_cross_views(S, T, vset);
    int16_t* maps = (int16_t*)malloc((size_t)nv * plane * sizeof(int16_t));
    uint64_t* cref = (uint64_t*)malloc(C * plane * sizeof(uint64_t));
    uint64_t* cview = (uint64_t*)malloc(plane * sizeof(uint64_t));
    int32_t* cost = (int32_t*)malloc(vol * sizeof(int32_t));
    int32_t* cpart = (int32_t*)malloc(vol * sizeof(int32_t));
    int64_t* csum = (int64_t*)malloc(vol * sizeof(int64_t));
    for (int ch = 0; ch < C; ++ch)
        census_of(prm, ref + ch * plane, H, W, cref + ch * plane);
    for (int i = 0; i < nv; ++i) {
        int s = vset[2 * i], t = vset[2 * i + 1];
        memset(cost, 0, vol * sizeof(int32_t));
        for (int ch = 0; ch < C; ++ch) {
            census_of(prm, views + (((size_t)t * S + s) * C + ch) * plane, H, W, cview);
            lfo_cost_census_view(cref + ch * plane, cview, H, W, sh - s, th - t, hyp, N, cpart);
            for (size_t e = 0; e < vol; ++e) cost[e] += cpart[e];
        }
        lfo_sgm(cost, NULL, NULL, H, W, N, prm->P1_init, prm->P2_init, prm->npaths, csum);
        lfo_wta(csum, NULL, NULL, H, W, N, maps + (size_t)i * plane);
        if (init_cost_out) memcpy(init_cost_out + (size_t)i * vol, cost, vol * sizeof(int32_t));
        if (init_csum_out) memcpy(init_csum_out + (size_t)i * vol, csum, vol * sizeof(int64_t));
    }
    free(cpart);

    /* fusion, hole filling, edges, borders (Sec. 3.4, Eq. 11) */
    int16_t* dinit = (int16_t*)malloc(plane * sizeof(int16_t));
    int16_t* tmp = (int16_t*)malloc(plane * sizeof(int16_t));
    lfo_fuse(maps, nv, H, W, prm->phi, dinit);
    for (int f = 0; f < prm->fill_passes; ++f) {
        lfo_fill(dinit, H, W, tmp);
        memcpy(dinit, tmp, plane * sizeof(int16_t));
    }
    uint8_t* edge = (uint8_t*)malloc(plane);
    lfo_edges(ref, C, H, W, prm->alpha, prm->edge_tau, edge);
    int16_t* lo = (int16_t*)malloc(plane * sizeof(int16_t));
    int16_t* hi = (int16_t*)malloc(plane * sizeof(int16_t));
    lfo_borders(dinit, edge, H, W, N, prm->lambda, prm->lambda_far, lo, hi);

    /* Sec. 3.5: bounded cost over all views (Eq. 12 or Eq. 15), bounded SGM, WTA */
    memset(cost, 0, vol * sizeof(int32_t));
    if (prm->cost_kind == 0) {
        float* s32 = (float*)malloc(vol * sizeof(float));
        lfo_cost_l2_f32(views, S, T, C, H, W, hyp, N, lo, hi, s32);
        lfo_quantize(s32, H, W, N, lo, hi, prm->alpha, prm->cost_cap, cost);
        free(s32);
    } else {
        uint64_t* call = (uint64_t*)malloc((size_t)S * T * C * plane * sizeof(uint64_t));
        for (int v = 0; v < S * T * C; ++v)
            census_of(prm, views + (size_t)v * plane, H, W, call + (size_t)v * plane);
        lfo_cost_census_all(call, S, T, C, H, W, hyp, N, lo, hi, prm->cost_cap, cost);
        free(call);
    }
    lfo_sgm(cost, lo, hi, H, W, N, prm->P1_final, prm->P2_final, prm->npaths, csum);
    int16_t* df = (int16_t*)malloc(plane * sizeof(int16_t));
    lfo_wta(csum, lo, hi, H, W, N, df);

    /* Sec. 3.6: sub-pixel parabola, then the median filter */
    float* dn = (float*)malloc(plane * sizeof(float));
    lfo_subpixel(csum, lo, hi, df, hyp, H, W, N, dn);
    if (prm->median == 3)
        lfo_median3(dn, H, W, disparity);
    else
        memcpy(disparity, dn, plane * sizeof(float));

    if (d_index) memcpy(d_index, df, plane * sizeof(int16_t));
    if (maps_out) memcpy(maps_out, maps, (size_t)nv * plane * sizeof(int16_t));
    if (dinit_out) memcpy(dinit_out, dinit, plane * sizeof(int16_t));
    if (lo_out) memcpy(lo_out, lo, plane * sizeof(int16_t));
    if (hi_out) memcpy(hi_out, hi, plane * sizeof(int16_t));
    if (cost_out) memcpy(cost_out, cost, vol * sizeof(int32_t));
    if (csum_out) memcpy(csum_out, csum, vol * sizeof(int64_t));

    free(maps); free(cref); free(cview); free(cost); free(csum); free(dinit); free(tmp);
    free(edge); free(lo); free(hi); free(df); free(dn);
    return 0;
}
