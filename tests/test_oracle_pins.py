"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a hand-derived
worked example, a closed form, an invariant, a textbook routine or brute force.
None of them needs a GPU.
"""
import itertools

import numpy as np
import pytest

import lfsynth
import oracle as lfo

rng = np.random.default_rng(12345)


# ------------------------------------------------------------------ Census
def test_census_constant_image_is_zero():
    # Eq. (3): equal values give xi = 0, so a constant image has all-zero strings.
    img = np.full((9, 11), 7.0, np.float32)
    assert not lfo.census(img, 7, 9).any()


def test_census_hand_example_and_bit_order():
    # Eq. (2)-(3), 3x3 window, row-major neighbour order with the centre skipped,
    # bit 0 first.  Centre 5 vs neighbours 1,2,3,4,6,7,8,9 -> 1,1,1,1,0,0,0,0.
    img = np.arange(1, 10, dtype=np.float32).reshape(3, 3)
    c = lfo.census(img, 3, 3)
    assert int(c[1, 1]) == 0b00001111
    # bottom-right corner 9 with clamp-to-edge neighbours
    # (5, 6, 6 | 8, 9 | 8, 9, 9): 9 > . gives 1,1,1,1,0,1,0,0
    assert int(c[2, 2]) == 0b00101111
    # top-left corner 1: nothing is smaller
    assert int(c[0, 0]) == 0


def test_census_window_bits_and_orientation():
    # a spike larger than everything sets all win_h*win_w - 1 bits (62 for 7x9)
    img = np.zeros((15, 15), np.float32)
    img[7, 7] = 1.0
    c = lfo.census(img, 7, 9)
    assert int(c[7, 7]) == (1 << 62) - 1
    # a pit (smaller than everything) sets none
    assert int(lfo.census(-img, 7, 9)[7, 7]) == 0
    # win_h counts rows: a 7x9 window sees 3 rows up and 4 columns left.  A single
    # smaller pixel 4 columns to the left of the centre, same row, sets bit 3*9+0 = 27.
    img = np.ones((15, 15), np.float32)
    img[7, 3] = 0.0
    assert int(lfo.census(img, 7, 9)[7, 7]) == 1 << 27
    # ... and 3 rows up, same column, sets bit 0*9+4 = 4
    img = np.ones((15, 15), np.float32)
    img[4, 7] = 0.0
    assert int(lfo.census(img, 7, 9)[7, 7]) == 1 << 4


def _window_offsets(win_h, win_w):
    # the dense window as a neighbour list: row-major, the centre skipped (Eq. 2)
    return [(i, j) for i in range(-(win_h // 2), win_h // 2 + 1)
            for j in range(-(win_w // 2), win_w // 2 + 1) if (i, j) != (0, 0)]


@pytest.mark.parametrize("win", [(3, 3), (5, 5), (7, 9), (1, 15), (9, 7)])
def test_sparse_census_with_the_whole_window_is_the_dense_census(win):
    # Sec. 3.2: a sparse window is a subset of the window's comparisons; with all
    # of them, in the dense order, it must be the dense Census, on images with
    # ties (8-bit values) and clamped borders.
    img = rng.integers(0, 6, size=(13, 17)).astype(np.float32)
    offs = _window_offsets(*win)
    assert np.array_equal(lfo.census(img, win[0], win[1], offsets=offs),
                          lfo.census(img, *win))


def test_sparse_census_bits_follow_the_list():
    # any subset of the window's offsets, in any order: bit n of the sparse string
    # is the dense string's bit of the n-th listed offset.  A swapped dy/dx (the
    # 7x9 window is not square), a flipped sign or an off-by-one order fails it.
    img = rng.integers(0, 9, size=(21, 23)).astype(np.float32)
    dense_list = _window_offsets(7, 9)
    dense = lfo.census(img, 7, 9)
    for trial in range(5):
        pick = rng.permutation(len(dense_list))[: int(rng.integers(1, len(dense_list) + 1))]
        offs = [dense_list[i] for i in pick]
        sparse = lfo.census(img, 7, 9, offsets=offs)
        want = np.zeros_like(dense)
        for n, i in enumerate(pick):
            want |= ((dense >> np.uint64(i)) & np.uint64(1)) << np.uint64(n)
        assert np.array_equal(sparse, want)


def test_sparse_census_hand_cases():
    img = np.array([[1, 5, 2],
                    [4, 3, 9],
                    [7, 0, 8]], np.float32)
    # one neighbour to the right: 1>5, 5>2, 2>2 (clamped) | 4>3, 3>9, 9>9 | 7>0, 0>8, 8>8
    c = lfo.census(img, 3, 3, offsets=[(0, 1)])
    assert c.astype(int).tolist() == [[0, 1, 0], [1, 0, 0], [1, 0, 0]]
    # the list order sets the bit order: below first, then left
    c = lfo.census(img, 3, 3, offsets=[(1, 0), (0, -1)])
    # centre 3: below 0 -> bit 0 = 1; left 4 -> bit 1 = 0
    assert int(c[1, 1]) == 0b01
    # centre 9: below 8 -> 1; left 3 -> 1
    assert int(c[1, 2]) == 0b11
    # centre 5 (top middle): below 3 -> 1; left 1 -> 1
    assert int(c[0, 1]) == 0b11
    # centre 7 (bottom left): below is itself (clamped) -> 0; left is itself -> 0
    assert int(c[2, 0]) == 0
    # 64 offsets, the most a string holds: a spike sets all 64 bits
    img = np.zeros((31, 31), np.float32)
    img[15, 15] = 1.0
    offs = [o for o in _window_offsets(15, 15) if (o[0] + o[1]) % 2 == 0][:64]
    assert len(offs) == 64
    assert int(lfo.census(img, 15, 15, offsets=offs)[15, 15]) == (1 << 64) - 1


def test_depth_with_the_whole_window_as_a_list_equals_the_dense_window():
    # the parameter path of lfo_depth: both stages' Census (initial, and Eq. (15)
    # as the final cost) take the list when one is given
    lf = lfsynth.workload("paper_s", seed=31, H=20, W=24, S=5, T=5, N=12)
    for kind in (0, 1):
        p = dict(lf.params, win_h=5, win_w=5, cost_kind=kind)
        a = lfo.depth(lf.views, lf.hyp, p, want_intermediates=True)
        b = lfo.depth(lf.views, lf.hyp, dict(p, census_offsets=_window_offsets(5, 5)),
                      want_intermediates=True)
        for k in ("maps", "dinit", "lo", "hi", "cost", "csum", "d_index", "disparity"):
            assert np.array_equal(a[k], b[k]), (kind, k)
        # a different list changes the result (the list is really used)
        c = lfo.depth(lf.views, lf.hyp, dict(p, census_offsets=[(0, 1), (1, 0)]),
                      want_intermediates=True)
        assert not np.array_equal(a["maps"], c["maps"])


def test_sparse_window_recovers_an_integer_plane():
    # a checkerboard 7x7 pattern (24 of the 48 comparisons) still finds the true
    # disparity of a fronto-parallel plane at an integer shift
    S = T = 5
    views = _shifted_lf(S, T, 36, 40, 1, seed=33)
    hyp = lfsynth.hypotheses(-2, 2, 17)
    prm = lfsynth._params(census=(7, 7), p_init=(10, 40), p_final=(10, 40))
    prm["census_offsets"] = lfsynth.checkerboard_census_offsets(7, 7)
    assert len(prm["census_offsets"]) == 24
    out = lfo.depth(views, hyp, prm)
    k = int(np.argmin(np.abs(hyp - 1)))
    assert (out["d_index"][8:-8, 8:-8] == k).all()


def test_hamming_matches_python_popcount():
    for _ in range(200):
        a, b = (int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64))
        a |= int(rng.integers(0, 2)) << 63
        assert lfo.hamming(a, b) == bin(a ^ b).count("1")
    assert lfo.hamming(0, (1 << 64) - 1) == 64


# -------------------------------------------------------------- cross views
def test_cross_views():
    # Sec. 3.4: the four cross-lying views, in the printed order
    assert lfo.cross_views(9, 9) == [(4, 0), (4, 8), (0, 4), (8, 4)]
    assert lfo.cross_views(5, 5) == [(2, 0), (2, 4), (0, 2), (4, 2)]
    # a horizontal 3-D light field: entries equal to the reference view drop out
    assert lfo.cross_views(11, 1) == [(0, 0), (10, 0)]
    assert lfo.cross_views(1, 7) == [(0, 0), (0, 6)]


# ---------------------------------------------------------- initial cost
def _shifted_lf(S, T, H, W, dstar, seed=0, margin=20):
    """Views of a fronto-parallel plane at integer disparity dstar: view (s,t) at
    pixel (x,y) shows reference pixel (x - (s_hat-s) dstar, y - (t_hat-t) dstar)."""
    r = np.random.default_rng(seed)
    big = r.integers(0, 256, size=(H + 2 * margin, W + 2 * margin)).astype(np.float32)
    sh, th = (S - 1) // 2, (T - 1) // 2
    views = np.empty((T, S, H, W), np.float32)
    for t in range(T):
        for s in range(S):
            ox = -(sh - s) * dstar
            oy = -(th - t) * dstar
            views[t, s] = big[margin + oy:margin + oy + H, margin + ox:margin + ox + W]
    return views


def test_initial_cost_constant_light_field_is_zero():
    views = np.full((5, 5, 12, 13), 0.3, np.float32)
    hyp = lfsynth.hypotheses(-2, 2, 9)
    c = lfo.census(views[2, 2], 5, 5)
    for (s, t) in lfo.cross_views(5, 5):
        cv = lfo.census(views[t, s], 5, 5)
        assert not lfo.cost_census_view(c, cv, 2 - s, 2 - t, hyp).any()


@pytest.mark.parametrize("dstar", [-2, 1])
def test_initial_cost_zero_at_true_integer_disparity(dstar):
    S = T = 5
    H, W = 24, 28
    views = _shifted_lf(S, T, H, W, dstar)
    hyp = lfsynth.hypotheses(-2, 2, 9)           # step 0.5: d = dstar is on the grid
    kstar = int(np.argmin(np.abs(hyp - dstar)))
    c = lfo.census(views[2, 2], 5, 5)
    m = 2 * abs(dstar) + 3                        # interior: no clamped tap, no clamped window
    for (s, t) in lfo.cross_views(S, T):
        cv = lfo.census(views[t, s], 5, 5)
        cost = lfo.cost_census_view(c, cv, 2 - s, 2 - t, hyp)
        assert not cost[m:-m, m:-m, kstar].any()
        # a wrong sign of the shift would not give zero: the mirrored hypothesis is not 0
        kmir = int(np.argmin(np.abs(hyp + dstar)))
        assert cost[m:-m, m:-m, kmir].mean() > 3


# ------------------------------------------------------------------- SGM
def _pairwise(a, b, P1, P2):
    return 0 if a == b else (P1 if abs(a - b) == 1 else P2)


def _path_lines(H, W, du, dv):
    """Pixels of every path line of direction (du, dv), in traversal order."""
    lines = []
    for v in range(H):
        for u in range(W):
            qu, qv = u - du, v - dv
            if 0 <= qu < W and 0 <= qv < H:
                continue                          # not a start pixel
            line = []
            x, y = u, v
            while 0 <= x < W and 0 <= y < H:
                line.append((y, x))
                x += du
                y += dv
            lines.append(line)
    return lines


def _brute_force_path(cost, lo, hi, du, dv, P1, P2):
    """L_r(p, k) = min over labellings of the path prefix ending at p with label k of
    sum C + sum V(k_i, k_i+1): exhaustive enumeration (exponential; tiny inputs)."""
    H, W, N = cost.shape
    L = np.full((H, W, N), -1, np.int64)
    for line in _path_lines(H, W, du, dv):
        labels = [range(lo[y, x], hi[y, x] + 1) for (y, x) in line]
        for n in range(1, len(line) + 1):
            y, x = line[n - 1]
            for k in labels[n - 1]:
                best = None
                for lab in itertools.product(*labels[:n - 1]):
                    lab = lab + (k,)
                    e = sum(int(cost[line[i][0], line[i][1], lab[i]]) for i in range(n))
                    e += sum(_pairwise(lab[i], lab[i + 1], P1, P2) for i in range(n - 1))
                    best = e if best is None or e < best else best
                L[y, x, k] = best
    return L


@pytest.mark.parametrize("ranged", [False, True])
@pytest.mark.parametrize("direction", [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1),
                                       (1, -1), (-1, 1),
                                       # the 8 more of the 16-path setting (Sec. 4.3)
                                       (1, 2), (-1, -2), (2, 1), (-2, -1), (2, -1), (-2, 1),
                                       (1, -2), (-1, 2)])
def test_sgm_path_equals_exhaustive_min_sum(direction, ranged):
    # Eq. (8) as printed is the min-sum dynamic programme along the path with
    # pairwise penalty 0 / P1 / P2 (P2 >= P1); checked by enumeration on paths of
    # at most 5 pixels and 4 labels, with and without per-pixel label ranges.
    H, W, N = 4, 5, 4
    P1, P2 = 3, 7
    cost = rng.integers(0, 12, size=(H, W, N)).astype(np.int32)
    if ranged:
        lo = rng.integers(0, N, size=(H, W)).astype(np.int16)
        hi = np.minimum(lo + rng.integers(0, 3, size=(H, W)), N - 1).astype(np.int16)
    else:
        lo = np.zeros((H, W), np.int16)
        hi = np.full((H, W), N - 1, np.int16)
    du, dv = direction
    ref = _brute_force_path(cost, lo, hi, du, dv, P1, P2)
    lit = lfo.sgm_path(cost, du, dv, P1, P2, lo=lo, hi=hi, literal=True)
    norm = lfo.sgm_path(cost, du, dv, P1, P2, lo=lo, hi=hi, literal=False)
    mask = np.zeros((H, W, N), bool)
    for y in range(H):
        for x in range(W):
            mask[y, x, lo[y, x]:hi[y, x] + 1] = True
    assert np.array_equal(lit[mask], ref[mask])
    # the normalised form differs from Eq. (8) by a per-pixel constant
    diff = np.where(mask, lit - norm, 0)
    for y in range(H):
        for x in range(W):
            d = diff[y, x, lo[y, x]:hi[y, x] + 1]
            assert (d == d[0]).all() and d[0] >= 0
    # invariant of the normalised form: 0 <= L_r <= C + P2
    assert (norm[mask] >= 0).all() and (norm[mask] <= cost[mask] + P2).all()


def test_sgm_zero_penalties_reduce_to_the_raw_cost():
    # P1 = P2 = 0: every term of the min equals m, so L_r = C and C_s = npaths * C.
    cost = rng.integers(0, 60, size=(7, 9, 6)).astype(np.int32)
    cs = lfo.sgm(cost, 0, 0, npaths=8)
    assert np.array_equal(cs, 8 * cost.astype(np.int64))
    assert np.array_equal(lfo.wta(cs), np.argmin(cost, axis=2).astype(np.int16))


def test_sgm_16_paths_sum_every_direction_once():
    # Eq. (9) over 16 directions: P1 = P2 = 0 gives 16 C; a single pixel is the
    # start of every path; and the set is closed under mirroring and transposition.
    cost = rng.integers(0, 60, size=(7, 9, 6)).astype(np.int32)
    assert np.array_equal(lfo.sgm(cost, 0, 0, npaths=16), 16 * cost.astype(np.int64))
    one = np.array([[[5, 2, 9]]], np.int32)
    assert np.array_equal(lfo.sgm(one, 3, 9, npaths=16)[0, 0], [80, 32, 144])
    c = rng.integers(0, 40, size=(6, 8, 5)).astype(np.int32)
    a = lfo.sgm(c, 4, 19, npaths=16)
    assert np.array_equal(lfo.sgm(c[:, ::-1].copy(), 4, 19, npaths=16), a[:, ::-1])
    assert np.array_equal(lfo.sgm(c[::-1].copy(), 4, 19, npaths=16), a[::-1])
    assert np.array_equal(lfo.sgm(c.transpose(1, 0, 2).copy(), 4, 19, npaths=16),
                          a.transpose(1, 0, 2))
    # the 16-path sum exceeds the 8-path one by the 8 knight-move paths, each >= 0
    assert (a >= lfo.sgm(c, 4, 19, npaths=8)).all()


def test_sgm_flip_equivariance():
    # The 8 directions are closed under mirroring: flipping the image flips C_s.
    cost = rng.integers(0, 40, size=(6, 8, 5)).astype(np.int32)
    a = lfo.sgm(cost, 4, 19)
    assert np.array_equal(lfo.sgm(cost[:, ::-1].copy(), 4, 19), a[:, ::-1])
    assert np.array_equal(lfo.sgm(cost[::-1].copy(), 4, 19), a[::-1])
    assert np.array_equal(lfo.sgm(cost.transpose(1, 0, 2).copy(), 4, 19), a.transpose(1, 0, 2))


def test_sgm_full_range_bounds_equal_dense():
    cost = rng.integers(0, 40, size=(6, 8, 5)).astype(np.int32)
    lo = np.zeros((6, 8), np.int16)
    hi = np.full((6, 8), 4, np.int16)
    assert np.array_equal(lfo.sgm(cost, 4, 19, lo=lo, hi=hi), lfo.sgm(cost, 4, 19))


def test_sgm_single_pixel_image():
    # every direction's path is the pixel alone: C_s = npaths * C
    cost = np.array([[[5, 2, 9]]], np.int32)
    assert np.array_equal(lfo.sgm(cost, 3, 9)[0, 0], [40, 16, 72])


def test_wta_ties_take_lowest_index():
    cs = np.array([[[5, 3, 3, 4], [2, 2, 2, 2], [9, 8, 7, 7]]], np.int64)
    assert lfo.wta(cs).tolist() == [[1, 0, 2]]
    lo = np.array([[2, 1, 0]], np.int16)
    hi = np.array([[3, 3, 1]], np.int16)
    assert lfo.wta(cs, lo, hi).tolist() == [[2, 1, 1]]


# --------------------------------------------------- fusion, fill, borders
def test_fusion_hand_cases():
    # D_init = D_1; average while |D_init - D_i| < phi, else invalid for good
    maps = np.array([[[10, 10, 10, 10, 0]],
                     [[12, 13, 10, 20, 1]],
                     [[11, 11, 30, 10, 0]],
                     [[11, 11, 10, 10, 2]]], np.int16)
    out = lfo.fuse(maps, 3)
    # px0: 10 -> (10+12)//2 = 11 -> (11+11)//2 = 11 -> 11
    # px1: |10-13| = 3 is not < 3 -> invalid
    # px2: 10 -> 10 -> |10-30| -> invalid (sticky, later agreement does not help)
    # px3: |10-20| -> invalid
    # px4: 0 -> (0+1)//2 = 0 -> 0 -> |0-2| < 3 -> 1
    assert out.tolist() == [[11, -1, -1, -1, 1]]


def test_fill_lower_median_and_jacobi():
    d = np.array([[4, 7, -1],
                  [-1, -1, 9],
                  [1, -1, -1]], np.int16)
    f = lfo.fill(d)
    # (0,2): valid neighbours 7, 9 -> lower median 7
    # (1,0): 4, 7, 1 -> 4;  (1,1): 4, 7, 9, 1 -> lower median of 1,4,7,9 = 4
    # (2,1): 1, 9 -> 1;  (2,2): 9 -> 9 (Jacobi: reads the input only)
    assert f.tolist() == [[4, 7, 7], [4, 4, 9], [1, 1, 9]]
    empty = np.full((3, 3), -1, np.int16)
    assert (lfo.fill(empty) == -1).all()


def test_edges_on_a_step():
    # a vertical step of height h: Gx = 4h on the two columns beside it, Gy = 0
    img = np.zeros((5, 6), np.float32)
    img[:, 3:] = 10.0
    e = lfo.edges(img, 1.0, 39.0)
    assert e[:, 2].all() and e[:, 3].all()
    assert not e[:, [0, 1, 4, 5]].any()
    assert not lfo.edges(img, 1.0, 40.0).any()           # 4h = 40 is not > 40
    assert lfo.edges(img / 255.0, 255.0, 39.0)[:, 2].all()  # alpha scales to 8-bit units
    assert not lfo.edges(img, 1.0, np.inf).any()


def test_borders_saturate_and_full_range():
    dinit = np.array([[0, 5, 9, -1]], np.int16)
    edge = np.array([[0, 0, 0, 0]], np.uint8)
    lo, hi = lfo.borders(dinit, edge, 10, 2)
    assert lo.tolist() == [[0, 3, 7, 0]] and hi.tolist() == [[2, 7, 9, 9]]
    edge[0, 1] = 1
    lo, hi = lfo.borders(dinit, edge, 10, 2)
    assert lo[0, 1] == 0 and hi[0, 1] == 9
    # lambda = -1: the boundary-less search of Sec. 4.5 keeps the full range everywhere
    edge[0, 1] = 0
    lo, hi = lfo.borders(dinit, edge, 10, -1)
    assert lo.tolist() == [[0, 0, 0, 0]] and hi.tolist() == [[9, 9, 9, 9]]


# ------------------------------------------------------------- l2 cost
def test_l2_identical_views_zero_at_zero_disparity():
    img = rng.random((10, 12)).astype(np.float32)
    views = np.broadcast_to(img, (3, 5, 10, 12)).copy()
    hyp = np.array([-1.0, 0.0, 0.5], np.float32)
    assert (lfo.cost_l2_f64(views, hyp)[:, :, 1] == 0).all()
    assert (lfo.cost_l2_f32(views, hyp)[:, :, 1] == 0).all()


@pytest.mark.parametrize("dstar", [-2, 1])
def test_l2_zero_at_true_integer_disparity(dstar):
    views = _shifted_lf(5, 5, 20, 22, dstar, seed=3) / 255.0
    hyp = lfsynth.hypotheses(-2, 2, 9)
    k = int(np.argmin(np.abs(hyp - dstar)))
    m = 2 * abs(dstar) + 1
    for f in (lfo.cost_l2_f64, lfo.cost_l2_f32):
        s = f(views, hyp)
        assert (s[m:-m, m:-m, k] == 0).all()
        assert (s[m:-m, m:-m, :].argmin(axis=2) == k).all()


@pytest.mark.parametrize("axis", ["u", "v"])
def test_l2_linear_ramp_closed_form(axis):
    # I(u, v) = a*u + b (or along v) on a fronto-parallel plane at non-integer d*:
    # view(s,t)(x) = a (x - cs d*) + b and bilinear sampling is exact on a linear
    # function, so S(d) = |a| |d - d*| * T * sum_s |s_hat - s| (for u; symmetric for v).
    S, T, H, W = 5, 3, 16, 40
    if axis == "v":
        S, T, H, W = 3, 5, 40, 16
    a, b, dstar = 0.01, 0.2, -0.7
    sh, th = (S - 1) // 2, (T - 1) // 2
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    views = np.empty((T, S, H, W), np.float32)
    for t in range(T):
        for s in range(S):
            if axis == "u":
                views[t, s] = a * (xx - (sh - s) * dstar) + b
            else:
                views[t, s] = a * (yy - (th - t) * dstar) + b
    hyp = np.array([-1.3, -0.7, -0.45, 0.2], np.float32)
    if axis == "u":
        closed = abs(a) * np.abs(hyp.astype(np.float64) - dstar) * T * sum(abs(sh - s) for s in range(S))
        sl = np.s_[:, 6:-6]
    else:
        closed = abs(a) * np.abs(hyp.astype(np.float64) - dstar) * S * sum(abs(th - t) for t in range(T))
        sl = np.s_[6:-6, :]
    s64 = lfo.cost_l2_f64(views, hyp)[sl]
    s32 = lfo.cost_l2_f32(views, hyp)[sl]
    np.testing.assert_allclose(s64, np.broadcast_to(closed, s64.shape), rtol=0, atol=5e-6)
    np.testing.assert_allclose(s32, np.broadcast_to(closed, s32.shape), rtol=0, atol=5e-5)


def test_l2_f32_within_rounding_of_f64():
    lf = lfsynth.workload("paper_s", H=24, W=28, S=5, T=5, N=16)
    s64 = lfo.cost_l2_f64(lf.views, lf.hyp)
    s32 = lfo.cost_l2_f32(lf.views, lf.hyp).astype(np.float64)
    # each of the S*T terms carries a few float32 roundings of values <= 1
    bound = lf.S * lf.T * 8 * 2.0 ** -24 + 1e-6 * s64
    assert (np.abs(s32 - s64) <= bound).all()


def test_quantize_round_half_even_and_cap():
    s = np.array([[[0.5, 1.5, 2.5, 3.49, 100.0]]], np.float32)
    q = lfo.quantize(s, 1.0, 50)
    assert q.tolist() == [[[0, 2, 2, 3, 50]]]


def test_cost_cap():
    assert lfo.cost_cap(35, 8, 32) == 65535 - 70
    assert lfo.cost_cap(120, 8, 16) == 65535 // 8 - 120
    assert lfo.cost_cap(120, 8, 16) + 2 * 120 <= 65535


def _path_cost_extremes(cost, P1, P2, npaths):
    """Largest path cost L_r over every direction and the largest sum C_s."""
    dirs = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1),
            (1, 2), (-1, -2), (2, 1), (-2, -1), (2, -1), (-2, 1), (1, -2), (-1, 2)][:npaths]
    lmax = max(int(lfo.sgm_path(cost, du, dv, P1, P2).max()) for du, dv in dirs)
    return lmax, int(lfo.sgm(cost, P1, P2, npaths).max())


@pytest.mark.parametrize("P2,npaths,sum_bits", [(35, 8, 32), (120, 8, 16), (250, 16, 16),
                                                (16383, 8, 32)])
def test_cost_cap_keeps_path_costs_and_sums_in_16_bits(P2, npaths, sum_bits):
    # What the cap is for (reading R9): with every cost <= cap, the normalised path
    # costs of Eq. (8) stay <= cap + P2 and leave room for the term m + P2 below a
    # 16-bit +inf of 65535; with 16-bit sums, Eq. (9) stays <= 65535.  Checked on
    # the oracle's own int64 path costs, on costs that sit at the cap with pits of
    # zero cost (the jumps that push a path cost up by P2).
    cap = lfo.cost_cap(P2, npaths, sum_bits)
    rng = np.random.default_rng(P2 + npaths)
    cost = np.full((9, 11, 6), cap, np.int32)
    pits = rng.random(cost.shape) < 0.3
    cost[pits] = rng.integers(0, cap + 1, size=int(pits.sum()))
    lmax, smax = _path_cost_extremes(cost, P1=min(7, P2), P2=P2, npaths=npaths)
    assert lmax <= cap + P2
    assert lmax + P2 <= 65535                      # m + P2 never passes the sentinel
    if sum_bits == 16:
        assert smax <= 65535
    # the bound L_r <= C + P2 is reached: a pixel at the cap after a zero-cost pit
    # (the cap could not be raised by P2 without breaking it)
    line = np.full((1, 2, 3), cap, np.int32)
    line[0, 0, 0] = 0
    L = lfo.sgm_path(line, 1, 0, P1=min(7, P2), P2=P2)
    assert L[0, 1, 2] == cap + P2


def test_initial_cost_rounds_half_pixel_shifts_to_even():
    # Eq. (7) samples the cross view at the nearest pixel of the Eq. (1) position;
    # a product (s_hat - s) d_k that is exactly x.5 goes to the even neighbour
    # (reading R2: rint, round half to even).  cview[x] holds x set bits and cref
    # none, so each cost is the column (or row) that was sampled.
    n = 16
    cref = np.zeros((1, n), np.uint64)
    cview = np.array([[(1 << x) - 1 for x in range(n)]], np.uint64)
    hyp = np.array([-2.5, -1.5, -0.5, 0.5, 1.5, 2.5], np.float32)
    u = 7
    cost = lfo.cost_census_view(cref, cview, 1, 0, hyp)
    assert cost[0, u].tolist() == [u + round(float(d)) for d in hyp]   # Python: half to even
    assert cost[0, u].tolist() == [5, 5, 7, 7, 9, 9]                   # half away: 4,5,6,8,9,10
    # the same along the vertical axis with t_hat - t = 3; the product is rounded to
    # float32 before rint: 3 * float32(1/6) is 0.50000001 in double precision (-> 1)
    # but exactly 0.5 in float32 (-> 0)
    cref_v = np.zeros((n, 1), np.uint64)
    cview_v = cview.reshape(n, 1)
    hyp_v = np.array([-0.5, 0.5, 1.0 / 6.0], np.float32)
    cost_v = lfo.cost_census_view(cref_v, cview_v, 0, 3, hyp_v)
    assert cost_v[u, 0].tolist() == [u - 2, u + 2, u]


def test_census_all_constant_and_integer_plane():
    views = _shifted_lf(3, 3, 20, 22, 1, seed=5)
    hyp = lfsynth.hypotheses(-2, 2, 9)
    call = np.stack([np.stack([lfo.census(views[t, s], 3, 3) for s in range(3)]) for t in range(3)])
    c = lfo.cost_census_all(call, hyp, 10**6)
    k = int(np.argmin(np.abs(hyp - 1)))
    assert (c[3:-3, 3:-3, k] == 0).all()
    const = np.zeros_like(call)
    assert not lfo.cost_census_all(const, hyp, 10**6).any()


# ----------------------------------------------------------- sub-pixel
def test_subpixel_is_the_parabola_vertex():
    # the vertex of the parabola through (-1,c-), (0,c0), (1,c+), found by a
    # least-squares fit (numpy.polyfit), must equal the offset the oracle applies
    hyp = np.linspace(-1, 1, 11).astype(np.float32)
    step = float(hyp[6] - hyp[5])
    for cm, c0, cp in [(10, 4, 6), (9, 1, 9), (7, 3, 20), (100, 60, 61)]:
        cs = np.zeros((1, 1, 11), np.int64) + 1000
        cs[0, 0, 4:7] = [cm, c0, cp]
        idx = np.array([[5]], np.int16)
        d = lfo.subpixel(cs, idx, hyp)[0, 0]
        A, B, _ = np.polyfit([-1.0, 0.0, 1.0], [cm, c0, cp], 2)
        vertex = -B / (2 * A)
        assert abs(vertex) <= 0.5
        assert abs((d - hyp[5]) / step - vertex) < 1e-5


def test_subpixel_validity_conditions():
    hyp = np.linspace(0, 1, 8).astype(np.float32)
    cs = np.array([[[9, 5, 2, 7, 9, 9, 9, 9]]], np.int64)
    idx = np.array([[2]], np.int16)
    # interior of [0,7], width ok -> refined
    assert lfo.subpixel(cs, idx, hyp)[0, 0] != hyp[2]
    # k* at the low border of its range -> no refinement
    lo, hi = np.array([[2]], np.int16), np.array([[7]], np.int16)
    assert lfo.subpixel(cs, idx, hyp, lo, hi)[0, 0] == hyp[2]
    # range [0,3]: interior [1,2] has only 2 indices (< 3) -> no refinement
    lo, hi = np.array([[0]], np.int16), np.array([[3]], np.int16)
    assert lfo.subpixel(cs, idx, hyp, lo, hi)[0, 0] == hyp[2]
    # range [0,4]: interior [1,3] has 3 indices -> refined
    hi = np.array([[4]], np.int16)
    assert lfo.subpixel(cs, idx, hyp, lo, hi)[0, 0] != hyp[2]


def test_median3_matches_scipy():
    from scipy.ndimage import median_filter
    x = rng.random((13, 17)).astype(np.float32)
    assert np.array_equal(lfo.median3(x), median_filter(x, size=3, mode="nearest"))


# ------------------------------------------------------------ end to end
def test_depth_recovers_integer_fronto_parallel_plane():
    # a fronto-parallel plane at an integer disparity, hypotheses on an integer-
    # compatible grid: the final index is the true one on interior pixels and the
    # refined disparity stays within half a step of it.
    S = T = 5
    H, W = 40, 44
    dstar = 1
    views = _shifted_lf(S, T, H, W, dstar, seed=11)
    hyp = lfsynth.hypotheses(-2, 2, 17)            # step 0.25
    k = int(np.argmin(np.abs(hyp - dstar)))
    prm = lfsynth._params()
    out = lfo.depth(views, hyp, prm, want_intermediates=True)
    m = 2 * 2 + 4
    assert (out["d_index"][m:-m, m:-m] == k).all()
    assert (np.abs(out["disparity"][m:-m, m:-m] - dstar) <= 0.125).all()
    # The initial maps use nearest-pixel shifts (Census cannot be interpolated):
    # every hypothesis whose rounded shift on the outer cross views (|s_hat-s| = 2)
    # equals the true one ties with it, and the lowest such index wins.
    shifts = np.rint(np.float32(2) * hyp)
    k_init = int(np.nonzero(shifts == 2 * dstar)[0].min())
    assert k_init < k
    assert (out["maps"][:, m:-m, m:-m] == k_init).all()


def test_boundless_search_equals_bounds_wider_than_the_range():
    # Sec. 4.5's boundary-less search and a border half-width lambda >= N - 1 give
    # every pixel the full range T, so the final stage -- and the map -- agree; and
    # the boundary-less map still recovers an integer fronto-parallel plane.
    S = T = 5
    H, W = 30, 34
    views = _shifted_lf(S, T, H, W, 1, seed=12)
    hyp = lfsynth.hypotheses(-2, 2, 17)
    wide = lfsynth._params(lam=16)
    free = lfsynth._params(lam=-1)
    a = lfo.depth(views, hyp, wide, want_intermediates=True)
    b = lfo.depth(views, hyp, free, want_intermediates=True)
    assert (b["lo"] == 0).all() and (b["hi"] == 16).all()
    assert np.array_equal(a["lo"], b["lo"]) and np.array_equal(a["hi"], b["hi"])
    assert np.array_equal(a["disparity"], b["disparity"])
    k = int(np.argmin(np.abs(hyp - 1)))
    m = 8
    assert (b["d_index"][m:-m, m:-m] == k).all()


# ------------------------------------------------ adaptive borders (Sec. 4.6)
def test_adaptive_border_width_hand_cases():
    # lambda_far at k = 0 (the farthest point) down to lambda at k = N-1, linear in
    # the index, rounded half up; lambda_far <= lambda keeps lambda everywhere
    N = 101
    assert [lfo.border_width(3, 7, d, N) for d in (0, 25, 50, 87, 88, 100)] == [7, 6, 5, 4, 3, 3]
    assert [lfo.border_width(3, 3, d, N) for d in (0, 50, 100)] == [3, 3, 3]
    assert [lfo.border_width(3, 2, d, N) for d in (0, 100)] == [3, 3]
    dinit = np.array([[0, 50, 100, -1]], np.int16)
    lo, hi = lfo.borders(dinit, None, N, 3, 7)
    assert lo.tolist() == [[0, 45, 97, 0]] and hi.tolist() == [[7, 55, 100, 100]]


def test_adaptive_borders_contain_the_constant_ones():
    # a wider border never drops a hypothesis the constant one keeps
    rng_ = np.random.default_rng(3)
    dinit = rng_.integers(-1, 64, size=(9, 11)).astype(np.int16)
    lo0, hi0 = lfo.borders(dinit, None, 64, 2)
    lo1, hi1 = lfo.borders(dinit, None, 64, 2, 9)
    assert (lo1 <= lo0).all() and (hi1 >= hi0).all()


# ------------------------------------------------------- colour (Sec. 3.2)
def test_colour_census_cost_sums_the_channels():
    # three identical channels: every Hamming distance counts three times
    S = T = 3
    views = _shifted_lf(S, T, 14, 17, 1, seed=4)
    hyp = lfsynth.hypotheses(-2, 2, 9)
    gray = np.stack([[lfo.census(views[t, s], 5, 5) for s in range(S)] for t in range(T)])
    colour = np.stack([gray] * 3, axis=2)                        # [T][S][C][H][W]
    a = lfo.cost_census_all(gray, hyp, 1 << 20)
    b = lfo.cost_census_all(colour, hyp, 1 << 20)
    assert np.array_equal(b, 3 * a)


def test_colour_l2_with_constant_extra_channels_equals_gray():
    # channels (g, c1, c2) with c1, c2 constant in every view: their differences are
    # exactly 0 and sqrt(x*x) == |x| in IEEE arithmetic, so the colour cost is the
    # gray one bit for bit (float32) and to the last place (float64)
    views = _shifted_lf(3, 5, 18, 21, -1, seed=5) / 255.0
    colour = np.stack([views, np.full_like(views, 0.25), np.full_like(views, 0.75)], axis=2)
    hyp = np.array([-1.6, -1.0, -0.35, 0.8], np.float32)
    assert np.array_equal(lfo.cost_l2_f32(colour, hyp), lfo.cost_l2_f32(views, hyp))
    assert np.array_equal(lfo.cost_l2_f64(colour, hyp), lfo.cost_l2_f64(views, hyp))


def test_colour_l2_linear_ramp_closed_form():
    # channel c is a_c*u + b_c on a plane at d*: every view's colour difference is
    # (s_hat-s)(d - d*) * (a_0, a_1, a_2), so S(d) = |a| |d - d*| T sum_s |s_hat-s|
    S, T, H, W = 5, 3, 16, 40
    a = np.array([0.01, -0.004, 0.007])
    b = np.array([0.2, 0.6, 0.4])
    dstar = 0.3
    sh = (S - 1) // 2
    xx = np.broadcast_to(np.arange(W, dtype=np.float64), (H, W))
    views = np.empty((T, S, 3, H, W), np.float32)
    for t in range(T):
        for s in range(S):
            for c in range(3):
                views[t, s, c] = a[c] * (xx - (sh - s) * dstar) + b[c]
    hyp = np.array([-1.1, 0.3, 0.55, 1.2], np.float32)
    closed = np.linalg.norm(a) * np.abs(hyp.astype(np.float64) - dstar) * T * \
        sum(abs(sh - s) for s in range(S))
    s64 = lfo.cost_l2_f64(views, hyp)[:, 6:-6]
    s32 = lfo.cost_l2_f32(views, hyp)[:, 6:-6]
    np.testing.assert_allclose(s64, np.broadcast_to(closed, s64.shape), rtol=0, atol=5e-6)
    np.testing.assert_allclose(s32, np.broadcast_to(closed, s32.shape), rtol=0, atol=5e-5)


def test_colour_depth_recovers_integer_plane_and_gray_channels_match_gray_maps():
    S = T = 5
    H, W = 36, 40
    g = _shifted_lf(S, T, H, W, 1, seed=13)
    r = _shifted_lf(S, T, H, W, 1, seed=14)
    colour = np.stack([g, r, 255.0 - g], axis=2)
    hyp = lfsynth.hypotheses(-2, 2, 17)
    prm = lfsynth._params(census=(3, 3), p_init=(10, 40), p_final=(10, 40))
    out = lfo.depth(colour, hyp, prm, want_intermediates=True)
    k = int(np.argmin(np.abs(hyp - 1)))
    m = 8
    assert (out["d_index"][m:-m, m:-m] == k).all()
    # the Sobel mask of identical channels is the gray one
    e1 = lfo.edges(g[2, 2], 1.0, 200.0)
    e3 = lfo.edges(np.stack([g[2, 2]] * 3), 1.0, 200.0)
    assert np.array_equal(e1, e3)
