"""The C-ABI library loads, exports every entry point include/lf.h declares, and
rejects invalid arguments on the host before touching the GPU (no compute call
runs here: every call below fails validation or is a pure host utility)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lf.h")


@pytest.fixture(scope="module")
def lf():
    from paper_1907_13449_amd import lf as binding
    return binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_six_calls_and_helpers():
    names = declared_functions()
    for n in ("lf_census", "lf_initial_disparity", "lf_cost_volume_bounded", "lf_sgm_aggregate",
              "lf_wta_subpixel", "lf_depth"):
        assert n in names


def _doc_before(text, name):
    # the comment block that precedes the declaration of `name`
    i = text.index(name + "(")
    j = text.rindex("/*", 0, i)
    lines = [ln.strip().lstrip("*").strip() for ln in text[j:i].splitlines()]
    return " ".join(" ".join(lines).split())


def test_header_states_the_bounds_contract():
    # lf_sgm_aggregate and lf_wta_subpixel read device-side bounds and offsets that
    # the host cannot check: their contract (and what the kernels do on a breach)
    # is part of the interface
    text = open(HEADER).read()
    agg = _doc_before(text, "lf_status lf_sgm_aggregate")
    assert "0 <= d_lo[p] <= d_hi[p] < N" in agg
    assert "exclusive prefix sum of d_hi - d_lo + 1" in agg
    assert "clamp the count to H*W*N" in agg
    wta = _doc_before(text, "lf_status lf_wta_subpixel")
    assert "Bounds contract as for lf_sgm_aggregate" in wta
    assert "clamped" in wta


def test_library_exports_every_declared_symbol(lf):
    for name in declared_functions():
        assert hasattr(lf.lib, name), name
    assert set(declared_functions()) == set(lf.EXPORTS)
    assert lf.lib.lf_abi_version() == 6


def test_struct_layouts_match_header(lf):
    # lf_view_set: pointer + 7 int32 (+ 4 bytes of tail padding);
    # lf_census_window: 3 int32 + 2 x 64 int8;
    # lf_params: the window + 3 + 3 + 3 int32 + 2 float + 4 int32
    assert C.sizeof(lf.ViewSet) == 8 + 7 * 4 + 4
    assert C.sizeof(lf.CensusWindow) == 3 * 4 + 2 * 64
    assert C.sizeof(lf.Params) == C.sizeof(lf.CensusWindow) + (3 + 3 + 3) * 4 + 2 * 4 + 4 * 4
    # lf_tuning: 6 int32
    assert C.sizeof(lf.Tuning) == 6 * 4


def test_validate_hypotheses(lf):
    lf.validate_hypotheses(np.linspace(-4, 4, 100, dtype=np.float32))
    with pytest.raises(lf.LFError):
        lf.validate_hypotheses(np.array([0.0, 0.0, 1.0], np.float32))
    with pytest.raises(lf.LFError):
        lf.validate_hypotheses(np.array([0.0], np.float32))
    with pytest.raises(lf.LFError):
        lf.validate_hypotheses(np.array([0.0, np.nan], np.float32))
    with pytest.raises(lf.LFError):
        lf.validate_hypotheses(np.linspace(0, 1, 257, dtype=np.float32))


def test_cross_views_and_cost_cap(lf):
    assert lf.cross_views(9, 9) == [(4, 0), (4, 8), (0, 4), (8, 4)]
    assert lf.cross_views(11, 1) == [(0, 0), (10, 0)]
    assert lf.cost_cap(35, 8, 32) == 65535 - 70
    assert lf.cost_cap(120, 8, 16) == 65535 // 8 - 120


def _params(lf, **kw):
    import lfsynth
    p = lfsynth._params()
    p.update(kw)
    return lf.make_params(p)


@pytest.mark.parametrize("bad", [
    dict(S=4, T=5), dict(S=1, T=1), dict(N=1), dict(N=300), dict(H=0), dict(C=2), dict(C=4),
    dict(H=2, W=65537), dict(H=65537, W=2),
])
def test_initial_disparity_rejects_bad_shapes(lf, bad):
    shape = dict(S=5, T=5, H=16, W=16, N=8, C=1)
    shape.update(bad)
    vs = lf.ViewSet(0x1000, shape["S"], shape["T"], shape["H"], shape["W"], shape["W"], lf.LF_U8,
                    shape["C"])
    prm = _params(lf)
    st = lf.lib.lf_initial_disparity(C.byref(vs), C.c_void_p(0x1000), shape["N"], C.byref(prm),
                                     None, C.c_void_p(0x1000), C.c_void_p(0x1000),
                                     C.c_void_p(0x1000), None, None, C.c_void_p(0x1000),
                                     1 << 30, None)
    assert st in (lf.LF_EINVAL, lf.LF_EUNSUPPORTED)
    assert lf.lib.lf_last_error()


@pytest.mark.parametrize("bad", [
    dict(win_h=4), dict(win_h=9, win_w=9), dict(win_h=17, win_w=3), dict(P1_init=50, P2_init=40),
    dict(npaths=4), dict(phi=0), dict(lam=-2), dict(median=5), dict(sum_bits=8),
    dict(cost_kind=7), dict(P2_init=9000), dict(lam_far=-1),
])
def test_params_rejected(lf, bad):
    vs = lf.ViewSet(0x1000, 5, 5, 16, 16, 16, lf.LF_U8, 1)
    prm = _params(lf, **bad)
    st = lf.lib.lf_depth(C.byref(vs), C.c_void_p(0x1000), 8, C.byref(prm), C.c_void_p(0x1000),
                         None, C.c_void_p(0x1000), 1 << 40, None)
    assert st in (lf.LF_EINVAL, lf.LF_EUNSUPPORTED)


def _depth_status(lf, prm):
    # a workspace too small for anything: LF_ENOSPACE once the parameters pass
    vs = lf.ViewSet(0x1000, 5, 5, 16, 16, 16, lf.LF_U8, 1)
    return lf.lib.lf_depth(C.byref(vs), C.c_void_p(0x1000), 8, C.byref(prm), C.c_void_p(0x1000),
                           None, C.c_void_p(0x1000), 1024, None)


@pytest.mark.parametrize("win,offsets", [
    ((5, 5), [(0, 0)]),                       # the centre
    ((5, 5), [(3, 0)]),                       # outside the bounding window (rows)
    ((5, 5), [(1, 1), (0, -3)]),              # outside (columns)
    ((7, 9), [(0, 5)]),
    ((4, 5), [(1, 1)]),                       # even side
    ((17, 3), [(1, 1)]),                      # side > 15
])
def test_sparse_windows_rejected(lf, win, offsets):
    prm = _params(lf, win_h=win[0], win_w=win[1], census_offsets=offsets)
    assert _depth_status(lf, prm) in (lf.LF_EINVAL, lf.LF_EUNSUPPORTED)


def test_sparse_window_bit_count(lf):
    import lfsynth
    # 65 listed neighbours is one too many (set directly: the binding refuses it)
    prm = _params(lf, win_h=15, win_w=15)
    prm.census.n_offsets = 65
    assert _depth_status(lf, prm) == lf.LF_EINVAL
    prm.census.n_offsets = -1
    assert _depth_status(lf, prm) == lf.LF_EINVAL
    with pytest.raises(ValueError):
        lf.census_window(15, 15, [(0, 1)] * 65)
    # a 15 x 15 bounding window (224 pixels) is fine with 64 listed neighbours,
    # and so are repeated neighbours
    offs = lfsynth.checkerboard_census_offsets(15, 15)[:64]
    assert _depth_status(lf, _params(lf, win_h=15, win_w=15, census_offsets=offs)) == lf.LF_ENOSPACE
    assert _depth_status(lf, _params(lf, census_offsets=[(1, 1)] * 3)) == lf.LF_ENOSPACE
    # entries beyond n_offsets are ignored
    prm = _params(lf, census_offsets=[(1, 1)])
    prm.census.dy[5] = 100
    assert _depth_status(lf, prm) == lf.LF_ENOSPACE


def test_workspace_too_small_is_enospace(lf):
    vs = lf.ViewSet(0x1000, 5, 5, 16, 16, 16, lf.LF_U8, 1)
    prm = _params(lf)
    st = lf.lib.lf_depth(C.byref(vs), C.c_void_p(0x1000), 8, C.byref(prm), C.c_void_p(0x1000),
                         None, C.c_void_p(0x1000), 1024, None)
    assert st == lf.LF_ENOSPACE


def test_cost_volume_capacity_is_checked(lf):
    vs = lf.ViewSet(0x1000, 5, 5, 16, 16, 16, lf.LF_U8, 1)
    prm = _params(lf)
    p = C.c_void_p(0x1000)
    st = lf.lib.lf_cost_volume_bounded(C.byref(vs), p, 8, C.byref(prm), p, p, p, p,
                                       16 * 16 * 8 - 1, None, p, 1 << 30, None)
    assert st == lf.LF_ENOSPACE


def test_workspace_sizes_are_positive_and_monotone(lf):
    prm = _params(lf)
    a = lf.lib.lf_depth_workspace_size(5, 5, 1, 96, 96, 32, C.byref(prm))
    b = lf.lib.lf_depth_workspace_size(9, 9, 1, 512, 512, 100, C.byref(prm))
    c = lf.lib.lf_depth_workspace_size(9, 9, 3, 512, 512, 100, C.byref(prm))
    assert 0 < a < b < c
    assert lf.lib.lf_depth_workspace_size(9, 9, 2, 512, 512, 100, C.byref(prm)) == 0
    # 9x9x512^2, N=100: dominated by the initial stage's per-direction path costs
    # (8 directions x 4 cross views x 512*512 pixels, at least a byte per hypothesis)
    assert b > 8 * 4 * 512 * 512 * 100
