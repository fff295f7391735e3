"""Seeded light fields shared by the GPU tests: shapes, dtypes, hypothesis counts
and parameters chosen to reach every kernel variant and edge case (ragged
tiles, N at the lane boundaries and at its maximum, 3-D light fields, one-row
and one-column images, 16-bit path costs, the Census cost kind)."""
import numpy as np

import lfsynth


def case(name):
    if name == "small":                      # 5x5 x 96^2 u8, N=32
        return lfsynth.workload("small")
    if name == "f32_ragged":                 # 7x7 x 70x83 f32, N=100 (K=2 with a tail)
        return lfsynth.workload("paper_s", H=70, W=83, S=7, T=7, N=100)
    if name == "u8_n65":                     # N=65: one hypothesis in the last lane pair
        lf = lfsynth.workload("paper_s", seed=7, H=33, W=47, S=5, T=5, N=65)
        lf.views = np.clip(np.rint(lf.views * 255.0), 0, 255).astype(np.uint8)
        lf.params.update(alpha=1.0, edge_tau=60.0)
        return lf
    if name == "n256":                       # N = 256, the maximum (K = 4)
        lf = lfsynth.workload("paper_s", seed=8, H=24, W=31, S=3, T=3, N=256)
        lf.params.update(win_h=5, win_w=5, sum_bits=32)
        return lf
    if name == "stage_1x11":                 # horizontal 3-D light field, |V| = 2
        sc = lfsynth.slanted_scene(9, 40, 120, 0.0, 6.0, S=11, T=1)
        v, gt = lfsynth.render(sc, 11, 1)
        v = np.clip(np.rint(v * 255.0), 0, 255).astype(np.uint8)
        p = lfsynth._params(census=(7, 9), p_init=(21, 45), p_final=(17, 35), lam=3,
                            edge_tau=128.0, alpha=1.0, sum_bits=32)
        return lfsynth.LightField(v, lfsynth.hypotheses(0.0, 6.0, 48), gt, p)
    if name == "col_7x1":                    # vertical 3-D light field
        sc = lfsynth.slanted_scene(10, 90, 20, -2.0, 2.0, S=1, T=7)
        v, gt = lfsynth.render(sc, 1, 7)
        return lfsynth.LightField(v, lfsynth.hypotheses(-2.0, 2.0, 20), gt,
                                  lfsynth._params(alpha=255.0, lam=1, fill=1, sum_bits=16))
    if name == "one_row":                    # H = 1: every diagonal line has one pixel
        lf = lfsynth.workload("paper_s", seed=11, H=1, W=64, S=3, T=3, N=12)
        lf.params.update(win_h=3, win_w=3, lam=0, fill_passes=0)
        return lf
    if name == "one_col":
        lf = lfsynth.workload("paper_s", seed=12, H=50, W=1, S=3, T=3, N=9)
        lf.params.update(win_h=3, win_w=3, median=0, fill_passes=3)
        return lf
    if name == "u16_paths":                  # bits + P2 > 255: 16-bit path-cost storage
        lf = lfsynth.workload("paper_s", seed=14, H=37, W=45, S=5, T=5, N=70)
        lf.params.update(P1_init=60, P2_init=250)
        return lf
    if name == "u16_tail":                   # 16-bit path costs in packed rows of 56 bytes:
        lf = lfsynth.workload("paper_s", seed=24, H=31, W=43, S=5, T=5, N=28)   # the
        lf.params.update(P1_init=60, P2_init=250)  # staged copy-out ends each with 8 bytes
        return lf
    if name == "k3_u8":                      # K = 3 hypotheses per lane, 8-bit path costs
        lf = lfsynth.workload("paper_s", seed=25, H=23, W=29, S=3, T=3, N=150)
        lf.params.update(win_h=5, win_w=5)
        return lf
    if name == "k4_u16":                     # K = 4 with 16-bit path costs (512-byte rows)
        lf = lfsynth.workload("paper_s", seed=26, H=19, W=27, S=3, T=3, N=200)
        lf.params.update(P1_init=60, P2_init=250, sum_bits=32)
        return lf
    if name == "k3_u16":                     # K = 3 with 16-bit path costs (384-byte rows)
        lf = lfsynth.workload("paper_s", seed=27, H=21, W=25, S=3, T=3, N=150)
        lf.params.update(P1_init=60, P2_init=250, sum_bits=32)
        return lf
    if name == "census_cost":                # Eq. (15) as the final cost
        lf = lfsynth.workload("paper_s", seed=13, H=40, W=52, S=5, T=5, N=24)
        lf.params.update(cost_kind=1, win_h=5, win_w=5, sum_bits=16)
        return lf
    if name == "paths16":                    # 16 directions (Sec. 4.3), 32-bit sums
        lf = lfsynth.workload("paper_s", seed=15, H=41, W=53, S=7, T=7, N=70)
        lf.params.update(npaths=16)
        return lf
    if name == "paths16_u16":                # 16 directions, 16-bit sums, 16-bit path costs
        lf = lfsynth.workload("paper_s", seed=16, H=30, W=37, S=5, T=5, N=40)
        lf.params.update(npaths=16, sum_bits=16, P1_init=40, P2_init=230)
        return lf
    if name == "boundless":                  # lambda = -1: full range everywhere (Sec. 4.5)
        lf = lfsynth.workload("paper_s", seed=17, H=36, W=45, S=5, T=5, N=48)
        lf.params.update(lam=-1)
        return lf
    if name == "rgb_f32":                    # colour views (Sec. 3.3), l2 over colour
        return lfsynth.workload("paper_s", seed=18, H=38, W=45, S=5, T=5, N=48, channels=3)
    if name == "rgb_u8_census":              # colour u8, Census cost kind, 16-bit sums
        lf = lfsynth.workload("paper_s", seed=19, H=30, W=41, S=3, T=3, N=40, channels=3)
        lf.views = np.clip(np.rint(lf.views * 255.0), 0, 255).astype(np.uint8)
        lf.params.update(cost_kind=1, win_h=5, win_w=5, sum_bits=16, alpha=1.0,
                         edge_tau=60.0)
        return lf
    if name == "u8_inf_add":                 # 8-bit path costs, but B + 2 P2 > 255 + P1:
        # hypotheses past N carry +inf by an add, not through the padded cost rows
        lf = lfsynth.workload("paper_s", seed=21, H=29, W=37, S=5, T=5, N=99)
        lf.params.update(P1_init=10, P2_init=190)
        return lf
    if name == "fill_4":                     # four fill passes: fusion, fill and borders
        lf = lfsynth.workload("paper_s", seed=22, H=26, W=33, S=5, T=5, N=20)   # launched apart
        lf.params.update(fill_passes=4, phi=1)
        return lf
    if name == "fill_3_sparse":              # three fill passes over a sparse initial map
        lf = lfsynth.workload("paper_s", seed=23, H=27, W=35, S=5, T=5, N=20)   # (phi = 1):
        lf.params.update(fill_passes=3, phi=1)   # holes reach the image edges in every tile
        return lf
    if name == "adaptive":                   # depth-adaptive borders (Sec. 4.6)
        lf = lfsynth.workload("paper_s", seed=20, H=44, W=50, S=7, T=7, N=80)
        lf.params.update(lam=2, lam_far=6)
        return lf
    if name == "half_shifts":                # (s_hat - s) d_k = x.5 exactly for odd k: the
        # nearest-pixel shift of Eq. (7) is decided by rounding half to even
        sc = lfsynth.two_plane_scene(28, 40, 48, d_back=-1.25, d_front=1.25, S=5, T=5)
        v, gt = lfsynth.render(sc, 5, 5, dtype=np.uint8)
        return lfsynth.LightField(v, lfsynth.hypotheses(-2.0, 2.0, 17), gt, lfsynth._params())
    if name == "plenoptic_s":                # 15x15 views (224 in the l2 sum), d in [-1.5, 1.5],
        # N = 64, noise 0.01: the plenoptic shape of the large workload at reduced size
        return lfsynth.workload("paper_s", seed=4001, H=56, W=80, S=15, T=15, N=64,
                                d_min=-1.5, d_max=1.5, noise=0.01)
    if name == "sparse_7x7":                 # a sparse 7x7 Census window (Sec. 3.2, 4.3):
        lf = lfsynth.workload("paper_s", seed=32, H=44, W=53, S=7, T=7, N=60)   # 24 bits
        lf.params.update(win_h=7, win_w=7,
                         census_offsets=lfsynth.checkerboard_census_offsets(7, 7))
        return lf
    if name == "sparse_64_census":           # 64 listed neighbours in a 15x15 window, in a
        lf = lfsynth.workload("paper_s", seed=33, H=35, W=42, S=5, T=5, N=30)   # random
        lf.params.update(win_h=15, win_w=15, cost_kind=1, sum_bits=32,  # order; Eq. (15)
                         census_offsets=random_census_offsets(15, 15, 64, seed=33))  # final
        return lf
    if name == "sparse_rgb":                 # colour u8 views, a sparse 5x5 window on both
        lf = lfsynth.workload("paper_s", seed=34, H=29, W=38, S=5, T=5, N=36,   # stages
                              channels=3)     # (Census per channel, Eq. (15) final cost)
        lf.views = np.clip(np.rint(lf.views * 255.0), 0, 255).astype(np.uint8)
        lf.params.update(win_h=5, win_w=5, cost_kind=1, sum_bits=16, alpha=1.0, edge_tau=60.0,
                         census_offsets=lfsynth.checkerboard_census_offsets(5, 5))
        return lf
    if name == "n2_tiny":                    # N = 2, the fewest hypotheses; a 3x3 light
        lf = lfsynth.workload("paper_s", seed=35, H=13, W=70, S=3, T=3, N=2,    # field
                              d_min=-1.0, d_max=1.0)
        lf.params.update(win_h=3, win_w=3, lam=0, phi=1)
        return lf
    if name == "n3_16paths":                 # N = 3 with 16 paths and 16-bit sums
        lf = lfsynth.workload("paper_s", seed=36, H=17, W=22, S=3, T=3, N=3,
                              d_min=-1.0, d_max=1.0)
        lf.params.update(npaths=16, sum_bits=16, lam=1)
        return lf
    if name == "stage_s":                    # 1x11 u8 moving-stage light field, d in [0, 24],
        return lfsynth.workload("stage", H=270, W=480)   # N = 96, |V| = 2, shifts to 120 px
    raise KeyError(name)


def random_census_offsets(win_h, win_w, n, seed):
    """n distinct neighbours of the win_h x win_w window in a seeded random order."""
    rng = np.random.default_rng(seed)
    cells = [(i, j) for i in range(-(win_h // 2), win_h // 2 + 1)
             for j in range(-(win_w // 2), win_w // 2 + 1) if (i, j) != (0, 0)]
    return [cells[k] for k in rng.permutation(len(cells))[:n]]


CASES = ["small", "f32_ragged", "u8_n65", "n256", "stage_1x11", "col_7x1", "one_row", "one_col",
         "u16_paths", "census_cost", "paths16", "paths16_u16", "boundless", "rgb_f32",
         "rgb_u8_census", "adaptive", "u8_inf_add", "fill_4", "fill_3_sparse", "u16_tail", "k3_u8",
         "k4_u16", "k3_u16", "half_shifts", "plenoptic_s", "stage_s", "sparse_7x7",
         "sparse_64_census", "sparse_rgb", "n2_tiny", "n3_16paths"]


