"""Python access to the CPU oracle (``liblfo.so``, built from ``lfo.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark; the product path never imports it.  The
oracle is a plain single-threaded C implementation of the method of "Rapid
Light Field Depth Estimation with Semi-Global Matching"; every C function cites
the passage it follows (see ``lfo.h``).  This wrapper only marshals numpy
arrays; it computes nothing itself.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lfo.c")
_LIB_PATH = os.path.join(_HERE, "liblfo.so")
_lib = None

CFLAGS = ["-O3", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile lfo.c into liblfo.so with gcc (-O3 -ffp-contract=off)."""
    global _lib
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
        _lib = None
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("win_h", C.c_int), ("win_w", C.c_int),
                ("P1_init", C.c_int), ("P2_init", C.c_int),
                ("P1_final", C.c_int), ("P2_final", C.c_int),
                ("npaths", C.c_int), ("phi", C.c_int), ("lambda_", C.c_int),
                ("fill_passes", C.c_int), ("lambda_far", C.c_int), ("channels", C.c_int),
                ("edge_tau", C.c_float), ("alpha", C.c_float),
                ("cost_kind", C.c_int), ("median", C.c_int), ("cost_cap", C.c_int32),
                ("n_offsets", C.c_int), ("off_dy", C.c_int * 64), ("off_dx", C.c_int * 64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB_PATH)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i16(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int16)


# --------------------------------------------------------------------- stages
def census(img, win_h, win_w, offsets=None):
    """Census strings of one plane; offsets: a list of (dy, dx) neighbours (the
    sparse window), else the dense win_h x win_w window."""
    img = _f32(img)
    H, W = img.shape
    out = np.zeros((H, W), dtype=np.uint64)
    if offsets:
        dy, dx = _offsets(offsets)
        lib().lfo_census_offsets(_p(img), H, W, len(offsets), _p(dy), _p(dx), _p(out))
    else:
        lib().lfo_census(_p(img), H, W, win_h, win_w, _p(out))
    return out


def _offsets(offsets):
    o = np.asarray(offsets, dtype=np.int32).reshape(-1, 2)
    if not 1 <= o.shape[0] <= 64:
        raise ValueError("1..64 Census offsets")
    return np.ascontiguousarray(o[:, 0]), np.ascontiguousarray(o[:, 1])


def hamming(a, b):
    return lib().lfo_hamming(C.c_uint64(int(a)), C.c_uint64(int(b)))


def cross_views(S, T):
    out = (C.c_int * 8)()
    n = lib().lfo_cross_views(S, T, out)
    return [(out[2 * i], out[2 * i + 1]) for i in range(n)]


def cost_census_view(cref, cview, cs, ct, hyp):
    cref = np.ascontiguousarray(cref, dtype=np.uint64)
    cview = np.ascontiguousarray(cview, dtype=np.uint64)
    hyp = _f32(hyp)
    H, W = cref.shape
    N = hyp.shape[0]
    out = np.zeros((H, W, N), dtype=np.int32)
    lib().lfo_cost_census_view(_p(cref), _p(cview), H, W, int(cs), int(ct), _p(hyp), N, _p(out))
    return out


def sgm_path(cost, du, dv, P1, P2, lo=None, hi=None, literal=False):
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    H, W, N = cost.shape
    lo, hi = _i16(lo), _i16(hi)
    L = np.zeros((H, W, N), dtype=np.int64)
    lib().lfo_sgm_path(_p(cost), _p(lo), _p(hi), H, W, N, int(du), int(dv), int(P1), int(P2),
                       int(bool(literal)), _p(L))
    return L


def sgm(cost, P1, P2, npaths=8, lo=None, hi=None):
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    H, W, N = cost.shape
    lo, hi = _i16(lo), _i16(hi)
    out = np.zeros((H, W, N), dtype=np.int64)
    lib().lfo_sgm(_p(cost), _p(lo), _p(hi), H, W, N, int(P1), int(P2), int(npaths), _p(out))
    return out


def wta(csum, lo=None, hi=None):
    csum = np.ascontiguousarray(csum, dtype=np.int64)
    H, W, N = csum.shape
    lo, hi = _i16(lo), _i16(hi)
    out = np.zeros((H, W), dtype=np.int16)
    lib().lfo_wta(_p(csum), _p(lo), _p(hi), H, W, N, _p(out))
    return out


def fuse(maps, phi):
    maps = _i16(maps)
    nv, H, W = maps.shape
    out = np.zeros((H, W), dtype=np.int16)
    lib().lfo_fuse(_p(maps), nv, H, W, int(phi), _p(out))
    return out


def fill(d):
    d = _i16(d)
    H, W = d.shape
    out = np.zeros((H, W), dtype=np.int16)
    lib().lfo_fill(_p(d), H, W, _p(out))
    return out


def _views(views):
    """[T][S][H][W] grayscale or [T][S][C][H][W] colour -> (float32 array, T, S, C, H, W)."""
    views = _f32(views)
    if views.ndim == 4:
        T, S, H, W = views.shape
        return views, T, S, 1, H, W
    T, S, Cn, H, W = views.shape
    return views, T, S, Cn, H, W


def edges(ref, alpha, tau):
    """ref: [H][W] or [C][H][W]."""
    ref = _f32(ref)
    Cn = 1 if ref.ndim == 2 else ref.shape[0]
    H, W = ref.shape[-2:]
    out = np.zeros((H, W), dtype=np.uint8)
    lib().lfo_edges(_p(ref), Cn, H, W, C.c_float(alpha), C.c_float(tau), _p(out))
    return out


def borders(dinit, edge, N, lam, lam_far=0):
    dinit = _i16(dinit)
    H, W = dinit.shape
    edge = None if edge is None else np.ascontiguousarray(edge, dtype=np.uint8)
    lo = np.zeros((H, W), dtype=np.int16)
    hi = np.zeros((H, W), dtype=np.int16)
    lib().lfo_borders(_p(dinit), _p(edge), H, W, int(N), int(lam), int(lam_far), _p(lo), _p(hi))
    return lo, hi


def border_width(lam, lam_far, d, N):
    return lib().lfo_border_width(int(lam), int(lam_far), int(d), int(N))


def cost_l2_f64(views, hyp, lo=None, hi=None):
    views, T, S, Cn, H, W = _views(views)
    hyp = _f32(hyp)
    N = hyp.shape[0]
    out = np.zeros((H, W, N), dtype=np.float64)
    lib().lfo_cost_l2_f64(_p(views), S, T, Cn, H, W, _p(hyp), N, _p(_i16(lo)), _p(_i16(hi)),
                          _p(out))
    return out


def cost_l2_f32(views, hyp, lo=None, hi=None):
    views, T, S, Cn, H, W = _views(views)
    hyp = _f32(hyp)
    N = hyp.shape[0]
    out = np.zeros((H, W, N), dtype=np.float32)
    lib().lfo_cost_l2_f32(_p(views), S, T, Cn, H, W, _p(hyp), N, _p(_i16(lo)), _p(_i16(hi)),
                          _p(out))
    return out


def quantize(s, alpha, cap, lo=None, hi=None):
    s = _f32(s)
    H, W, N = s.shape
    out = np.zeros((H, W, N), dtype=np.int32)
    lib().lfo_quantize(_p(s), H, W, N, _p(_i16(lo)), _p(_i16(hi)), C.c_float(alpha),
                       C.c_int32(int(cap)), _p(out))
    return out


def cost_census_all(census_all, hyp, cap, lo=None, hi=None):
    """census_all: [T][S][H][W] or [T][S][C][H][W] uint64."""
    census_all = np.ascontiguousarray(census_all, dtype=np.uint64)
    if census_all.ndim == 4:
        T, S, H, W = census_all.shape
        Cn = 1
    else:
        T, S, Cn, H, W = census_all.shape
    hyp = _f32(hyp)
    N = hyp.shape[0]
    out = np.zeros((H, W, N), dtype=np.int32)
    lib().lfo_cost_census_all(_p(census_all), S, T, Cn, H, W, _p(hyp), N, _p(_i16(lo)),
                              _p(_i16(hi)), C.c_int32(int(cap)), _p(out))
    return out


def subpixel(csum, idx, hyp, lo=None, hi=None):
    csum = np.ascontiguousarray(csum, dtype=np.int64)
    H, W, N = csum.shape
    out = np.zeros((H, W), dtype=np.float32)
    lib().lfo_subpixel(_p(csum), _p(_i16(lo)), _p(_i16(hi)), _p(_i16(idx)), _p(_f32(hyp)),
                       H, W, N, _p(out))
    return out


def median3(d):
    d = _f32(d)
    H, W = d.shape
    out = np.zeros((H, W), dtype=np.float32)
    lib().lfo_median3(_p(d), H, W, _p(out))
    return out


def cost_cap(P2_final, npaths, sum_bits):
    """Quantisation cap of the final cost (see lfo_cost_cap)."""
    return lib().lfo_cost_cap(int(P2_final), int(npaths), int(sum_bits))


def depth(views, hyp, params, want_intermediates=False, want_initial_volumes=False):
    """The whole method (Sec. 3.3-3.6) on one light field; returns a dict.  With
    want_initial_volumes also init_cost ([|V|][H][W][N] int32, Eq. 7) and init_csum
    ([|V|][H][W][N] int64, Eq. 9) of the initial stage."""
    views, T, S, Cn, H, W = _views(views)
    hyp = _f32(hyp)
    N = hyp.shape[0]
    pr = params
    prm = _Params(pr["win_h"], pr["win_w"], pr["P1_init"], pr["P2_init"], pr["P1_final"],
                  pr["P2_final"], pr["npaths"], pr["phi"], pr["lam"], pr["fill_passes"],
                  pr.get("lam_far", 0), Cn,
                  pr["edge_tau"], pr["alpha"], pr["cost_kind"], pr["median"],
                  cost_cap(pr["P2_final"], pr["npaths"], pr["sum_bits"]))
    if pr.get("census_offsets"):
        dy, dx = _offsets(pr["census_offsets"])
        prm.n_offsets = len(dy)
        prm.off_dy[:len(dy)] = dy.tolist()
        prm.off_dx[:len(dx)] = dx.tolist()
    nv = len(cross_views(S, T))
    disp = np.zeros((H, W), dtype=np.float32)
    idx = np.zeros((H, W), dtype=np.int16)
    out = dict(disparity=disp, d_index=idx)
    args = [None] * 6
    if want_intermediates:
        out.update(maps=np.zeros((nv, H, W), dtype=np.int16), dinit=np.zeros((H, W), np.int16),
                   lo=np.zeros((H, W), np.int16), hi=np.zeros((H, W), np.int16),
                   cost=np.zeros((H, W, N), np.int32), csum=np.zeros((H, W, N), np.int64))
        args = [out[k] for k in ("maps", "dinit", "lo", "hi", "cost", "csum")]
    if want_initial_volumes:
        out.update(init_cost=np.zeros((nv, H, W, N), np.int32),
                   init_csum=np.zeros((nv, H, W, N), np.int64))
    args = args + [out.get("init_cost"), out.get("init_csum")]
    rc = lib().lfo_depth(_p(views), S, T, H, W, _p(hyp), N, C.byref(prm), _p(disp), _p(idx),
                         *[_p(a) for a in args])
    if rc != 0:
        raise ValueError("lfo_depth: invalid arguments")
    return out
