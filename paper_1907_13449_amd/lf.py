"""ctypes binding of liblf (include/lf.h): the same entry points, taking torch
tensors that live on the GPU.

This module only marshals arguments -- shapes, dtypes, data pointers and the
current HIP stream -- and raises on a non-zero status.  Every step of the method
runs in the HIP kernels of liblf.so; there is no fallback: if the library is
missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblf.so")

LF_OK, LF_EINVAL, LF_ENOSPACE, LF_EDEVICE, LF_EUNSUPPORTED = 0, -1, -2, -3, -4
LF_EBUSY, LF_ETIMEOUT, LF_ECANCELED = -5, -6, -7
LF_U8, LF_F32 = 0, 1
LF_COST_L2, LF_COST_CENSUS = 0, 1

EXPORTS = (
    "lf_abi_version", "lf_last_error", "lf_validate_hypotheses", "lf_cost_cap",
    "lf_cross_views", "lf_census", "lf_initial_workspace_size", "lf_initial_disparity",
    "lf_cost_workspace_size", "lf_cost_volume_bounded", "lf_sgm_workspace_size",
    "lf_sgm_aggregate",
    "lf_wta_workspace_size", "lf_wta_subpixel", "lf_depth_workspace_size", "lf_depth",
    "lf_depth_noalloc", "lf_profile_enable", "lf_profile_read", "lf_profile_stage_name",
    "lf_batch_workspace_size", "lf_plan_create", "lf_plan_autotune", "lf_plan_capture",
    "lf_plan_run", "lf_plan_launches", "lf_plan_tuning", "lf_plan_destroy",
    "lf_server_create", "lf_server_submit", "lf_server_wait", "lf_server_stats",
    "lf_server_destroy",
)


class LFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"liblf status {status}: {msg}")
        self.status = status


class ViewSet(C.Structure):
    _fields_ = [("data", C.c_void_p), ("S", C.c_int32), ("T", C.c_int32), ("H", C.c_int32),
                ("W", C.c_int32), ("pitch", C.c_int32), ("dtype", C.c_int32),
                ("channels", C.c_int32)]


MAX_CENSUS_BITS = 64


class CensusWindow(C.Structure):
    _fields_ = [("win_h", C.c_int32), ("win_w", C.c_int32), ("n_offsets", C.c_int32),
                ("dy", C.c_int8 * MAX_CENSUS_BITS), ("dx", C.c_int8 * MAX_CENSUS_BITS)]


def census_window(win_h, win_w, offsets=None) -> CensusWindow:
    """lf_census_window: the dense win_h x win_w window, or with `offsets` (a list
    of up to 64 (dy, dx) pairs inside it) the sparse window of those neighbours."""
    w = CensusWindow(win_h, win_w, 0)
    if offsets:
        if len(offsets) > MAX_CENSUS_BITS:
            raise ValueError(f"at most {MAX_CENSUS_BITS} Census offsets")
        w.n_offsets = len(offsets)
        for n, (dy, dx) in enumerate(offsets):
            w.dy[n], w.dx[n] = int(dy), int(dx)
    return w


class SgmParams(C.Structure):
    _fields_ = [("P1", C.c_int32), ("P2", C.c_int32), ("npaths", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("census", CensusWindow), ("sgm_init", SgmParams), ("sgm_final", SgmParams),
                ("phi", C.c_int32), ("lambda_", C.c_int32), ("fill_passes", C.c_int32),
                ("edge_tau", C.c_float), ("alpha", C.c_float), ("cost_kind", C.c_int32),
                ("median", C.c_int32), ("sum_bits", C.c_int32), ("lambda_far", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("views", ViewSet), ("hyp", C.c_void_p), ("N", C.c_int32), ("params", Params),
                ("disparity", C.c_void_p), ("d_index", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("cost_cells_per_thread", C.c_int32), ("cost_stride", C.c_int32),
                ("dense_prefetch", C.c_int32), ("bounded_prefetch", C.c_int32),
                ("bounded_lanes", C.c_int32), ("bounded_offsets", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("max_batch", C.c_int32),
                ("max_inflight", C.c_int32), ("max_queue", C.c_int32),
                ("group_ratio", C.c_int32), ("tuning", Tuning), ("large_bytes", C.c_int64),
                ("max_large", C.c_int32)]


class RequestInfo(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_admit", C.c_double), ("t_launch", C.c_double),
                ("t_done", C.c_double), ("batch", C.c_int64), ("batch_size", C.c_int32),
                ("status", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"liblf.so not built ({LIB_PATH}); run python -m paper_1907_13449_amd.build")
    lib = C.CDLL(LIB_PATH)
    lib.lf_last_error.restype = C.c_char_p
    for name in ("lf_initial_workspace_size", "lf_cost_workspace_size", "lf_wta_workspace_size",
                 "lf_depth_workspace_size", "lf_sgm_workspace_size"):
        getattr(lib, name).restype = C.c_size_t
    P, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    lib.lf_census.argtypes = [P, i32, i32, i32, i32, CensusWindow, P, P]
    lib.lf_initial_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, P]
    lib.lf_initial_disparity.argtypes = [P, P, i32, P, P, P, P, P, P, P, P, sz, P]
    lib.lf_cost_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, P]
    lib.lf_cost_volume_bounded.argtypes = [P, P, i32, P, P, P, P, P, i64, P, P, sz, P]
    lib.lf_sgm_workspace_size.argtypes = [i32, i32, i32, i32]
    lib.lf_sgm_aggregate.argtypes = [P, P, P, P, i32, i32, i32, SgmParams, i32, P, P, sz, P]
    lib.lf_wta_workspace_size.argtypes = [i32, i32]
    lib.lf_wta_subpixel.argtypes = [P, i32, P, P, P, i32, i32, P, i32, i32, P, P, P, sz, P]
    lib.lf_depth_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, P]
    lib.lf_depth.argtypes = [P, P, i32, P, P, P, P, sz, P]
    lib.lf_depth_noalloc.argtypes = [P, P, i32, P, P, P, P]
    lib.lf_validate_hypotheses.argtypes = [P, i32]
    lib.lf_cost_cap.argtypes = [i32, i32, i32]
    lib.lf_cross_views.argtypes = [i32, i32, P]
    lib.lf_profile_enable.argtypes = [i32]
    lib.lf_profile_read.argtypes = [P, P, i32]
    lib.lf_profile_stage_name.argtypes = [i32]
    lib.lf_profile_stage_name.restype = C.c_char_p
    lib.lf_batch_workspace_size.argtypes = [P, i32]
    lib.lf_batch_workspace_size.restype = sz
    lib.lf_plan_create.argtypes = [P, i32, P, sz, P, P, P]
    lib.lf_plan_autotune.argtypes = [P, P, i32, P]
    lib.lf_plan_capture.argtypes = [P]
    lib.lf_plan_run.argtypes = [P, P]
    lib.lf_plan_launches.argtypes = [P]
    lib.lf_plan_tuning.argtypes = [P, P]
    lib.lf_plan_destroy.argtypes = [P]
    lib.lf_plan_destroy.restype = None
    lib.lf_server_create.argtypes = [P, P]
    lib.lf_server_submit.argtypes = [P, P, P, P]
    lib.lf_server_wait.argtypes = [P, i64, C.c_double, P]
    lib.lf_server_stats.argtypes = [P, P, P, P, P]
    lib.lf_server_stats.restype = None
    lib.lf_server_destroy.argtypes = [P]
    lib.lf_server_destroy.restype = None
    return lib


lib = _load()


# ------------------------------------------------------------------ helpers
def _check(status):
    if status != LF_OK:
        raise LFError(status, lib.lf_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name}: expected a contiguous {dtype} CUDA tensor")
    return t


PARAM_KEYS = frozenset(("win_h", "win_w", "census_offsets", "P1_init", "P2_init", "P1_final",
                        "P2_final", "npaths", "phi", "lam", "fill_passes", "edge_tau", "alpha", "cost_kind",
                        "median", "sum_bits", "lam_far"))


def make_params(p: dict) -> Params:
    """lf_params from a dict of method parameters (the keys of lfsynth workloads).
    Unknown keys are an error, so that a misspelt parameter is not silently
    left at its default."""
    unknown = set(p) - PARAM_KEYS
    if unknown:
        raise KeyError(f"unknown method parameters: {sorted(unknown)}")
    return Params(census_window(p["win_h"], p["win_w"], p.get("census_offsets")),
                  SgmParams(p["P1_init"], p["P2_init"], p["npaths"]),
                  SgmParams(p["P1_final"], p["P2_final"], p["npaths"]),
                  p["phi"], p["lam"], p["fill_passes"], float(p["edge_tau"]), float(p["alpha"]),
                  p["cost_kind"], p["median"], p["sum_bits"], p.get("lam_far", 0))


def view_set(views: torch.Tensor) -> ViewSet:
    """lf_view_set of a [T][S][H][W] (grayscale) or [T][S][C][H][W] (colour)
    uint8/float32 tensor on the GPU."""
    if views.dim() not in (4, 5) or not views.is_cuda or not views.is_contiguous():
        raise ValueError("views: expected a contiguous [T][S]([C])[H][W] CUDA tensor")
    if views.dtype == torch.uint8:
        dt = LF_U8
    elif views.dtype == torch.float32:
        dt = LF_F32
    else:
        raise ValueError("views: uint8 or float32")
    T, S = views.shape[:2]
    H, W = views.shape[-2:]
    channels = 1 if views.dim() == 4 else views.shape[2]
    return ViewSet(views.data_ptr(), S, T, H, W, W, dt, channels)


def workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(int(nbytes), 256)]


def cross_views(S, T):
    buf = (C.c_int32 * 8)()
    n = lib.lf_cross_views(S, T, buf)
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(n)]


def cost_cap(P2_final, npaths, sum_bits):
    return lib.lf_cost_cap(P2_final, npaths, sum_bits)


def validate_hypotheses(hyp_host) -> None:
    import numpy as np
    h = np.ascontiguousarray(hyp_host, dtype=np.float32)
    _check(lib.lf_validate_hypotheses(h.ctypes.data_as(C.c_void_p), h.shape[0]))


# ------------------------------------------------------------- entry points
def lf_census(img: torch.Tensor, win_h: int, win_w: int, out=None, stream=None,
              offsets=None):
    if img.dim() != 2 or not img.is_cuda or not img.is_contiguous():
        raise ValueError("img: contiguous [H][W] CUDA tensor")
    dt = LF_U8 if img.dtype == torch.uint8 else LF_F32
    if img.dtype not in (torch.uint8, torch.float32):
        raise ValueError("img: uint8 or float32")
    H, W = img.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.int64, device=img.device)
    _check(lib.lf_census(_ptr(img), dt, H, W, W, census_window(win_h, win_w, offsets), _ptr(out),
                         _stream(stream)))
    return out


def lf_initial_disparity(views: torch.Tensor, hyp: torch.Tensor, params: dict, want_maps=True,
                         want_volumes=False, ws=None, stream=None):
    """D_i per cross view, d_init, d_lo, d_hi; with want_volumes also the Census cost
    volume of Eq. (7) ([|V|][H][W][N] uint8) and the aggregated cost of Eq. (9)
    ([|V|][H][W][N], int16 tensor holding uint16 values)."""
    vs = view_set(views)
    prm = make_params(params)
    _dev(hyp, torch.float32, "hyp")
    N = hyp.shape[0]
    dev = views.device
    H, W = vs.H, vs.W
    nv = len(cross_views(vs.S, vs.T))
    maps = torch.empty((nv, H, W), dtype=torch.int16, device=dev) if want_maps else None
    d_init = torch.empty((H, W), dtype=torch.int16, device=dev)
    d_lo = torch.empty((H, W), dtype=torch.int16, device=dev)
    d_hi = torch.empty((H, W), dtype=torch.int16, device=dev)
    ccv = csum = None
    if want_volumes:
        ccv = torch.empty((nv, H, W, N), dtype=torch.uint8, device=dev)
        csum = torch.empty((nv, H, W, N), dtype=torch.int16, device=dev)
    need = lib.lf_initial_workspace_size(vs.S, vs.T, vs.channels, H, W, N, C.byref(prm))
    if ws is None:
        ws = workspace(need, dev)
    _check(lib.lf_initial_disparity(C.byref(vs), _ptr(hyp), N, C.byref(prm), _ptr(maps),
                                    _ptr(d_init), _ptr(d_lo), _ptr(d_hi), _ptr(ccv), _ptr(csum),
                                    _ptr(ws), ws.numel(), _stream(stream)))
    return dict(maps=maps, d_init=d_init, d_lo=d_lo, d_hi=d_hi, census_cost=ccv,
                csum_init=csum)


def lf_cost_volume_bounded(views: torch.Tensor, hyp: torch.Tensor, params: dict,
                           d_lo: torch.Tensor, d_hi: torch.Tensor, want_f32=False, ws=None,
                           stream=None, cap_cells=None):
    vs = view_set(views)
    prm = make_params(params)
    _dev(hyp, torch.float32, "hyp")
    _dev(d_lo, torch.int16, "d_lo")
    _dev(d_hi, torch.int16, "d_hi")
    N = hyp.shape[0]
    dev = views.device
    HW = vs.H * vs.W
    cells = HW * N if cap_cells is None else int(cap_cells)
    offsets = torch.empty(HW + 1, dtype=torch.int64, device=dev)
    cost = torch.empty(cells, dtype=torch.int16, device=dev)        # uint16 bits
    cost_f32 = torch.empty(cells, dtype=torch.float32, device=dev) if want_f32 else None
    need = lib.lf_cost_workspace_size(vs.S, vs.T, vs.channels, vs.H, vs.W, N, C.byref(prm))
    if ws is None:
        ws = workspace(need, dev)
    _check(lib.lf_cost_volume_bounded(C.byref(vs), _ptr(hyp), N, C.byref(prm), _ptr(d_lo),
                                      _ptr(d_hi), _ptr(offsets), _ptr(cost), cells,
                                      _ptr(cost_f32), _ptr(ws), ws.numel(), _stream(stream)))
    return dict(offsets=offsets, cost=cost, cost_f32=cost_f32)


def lf_sgm_aggregate(cost: torch.Tensor, offsets: torch.Tensor, d_lo: torch.Tensor,
                     d_hi: torch.Tensor, N: int, P1: int, P2: int, npaths: int = 8,
                     sum_bits: int = 32, csum=None, ws=None, stream=None):
    _dev(cost, torch.int16, "cost")
    _dev(offsets, torch.int64, "offsets")
    _dev(d_lo, torch.int16, "d_lo")
    _dev(d_hi, torch.int16, "d_hi")
    H, W = d_lo.shape
    if csum is None:
        csum = torch.empty(cost.numel(), dtype=torch.int16 if sum_bits == 16 else torch.int32,
                           device=cost.device)
    if ws is None:
        ws = workspace(lib.lf_sgm_workspace_size(H, W, N, npaths), cost.device)
    _check(lib.lf_sgm_aggregate(_ptr(cost), _ptr(offsets), _ptr(d_lo), _ptr(d_hi), H, W, N,
                                SgmParams(P1, P2, npaths), sum_bits, _ptr(csum), _ptr(ws),
                                ws.numel(), _stream(stream)))
    return csum


def lf_wta_subpixel(csum: torch.Tensor, sum_bits: int, offsets: torch.Tensor, d_lo: torch.Tensor,
                    d_hi: torch.Tensor, hyp: torch.Tensor, median: int = 3, ws=None, stream=None):
    H, W = d_lo.shape
    dev = csum.device
    d_index = torch.empty((H, W), dtype=torch.int16, device=dev)
    disp = torch.empty((H, W), dtype=torch.float32, device=dev)
    if ws is None:
        ws = workspace(lib.lf_wta_workspace_size(H, W), dev)
    _check(lib.lf_wta_subpixel(_ptr(csum), sum_bits, _ptr(offsets), _ptr(d_lo), _ptr(d_hi), H,
                               W, _ptr(hyp), hyp.shape[0], median, _ptr(d_index), _ptr(disp),
                               _ptr(ws), ws.numel(), _stream(stream)))
    return dict(d_index=d_index, disparity=disp)


def profile_enable(on: bool = True) -> bool:
    """Turn per-stage HIP-event timing on/off; returns the previous setting."""
    return bool(lib.lf_profile_enable(int(on)))


def profile_read():
    """{stage name: (milliseconds, launches)} accumulated since the last read."""
    n = 16
    ms = (C.c_double * n)()
    la = (C.c_int64 * n)()
    k = lib.lf_profile_read(ms, la, n)
    return {lib.lf_profile_stage_name(i).decode(): (ms[i], la[i]) for i in range(k)}


def depth_workspace_bytes(S, T, H, W, N, params: dict, channels: int = 1) -> int:
    prm = make_params(params)
    return lib.lf_depth_workspace_size(S, T, channels, H, W, N, C.byref(prm))


def lf_depth(views: torch.Tensor, hyp: torch.Tensor, params: dict, ws=None, out=None,
             d_index=None, stream=None):
    vs = view_set(views)
    prm = make_params(params)
    _dev(hyp, torch.float32, "hyp")
    N = hyp.shape[0]
    dev = views.device
    if out is None:
        out = torch.empty((vs.H, vs.W), dtype=torch.float32, device=dev)
    if ws is None:
        ws = workspace(lib.lf_depth_workspace_size(vs.S, vs.T, vs.channels, vs.H, vs.W, N,
                                                   C.byref(prm)), dev)
    _check(lib.lf_depth(C.byref(vs), _ptr(hyp), N, C.byref(prm), _ptr(out), _ptr(d_index),
                        _ptr(ws), ws.numel(), _stream(stream)))
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20      # LF_NOALLOC_SCRATCH_BYTES


def lf_depth_noalloc(views: torch.Tensor, hyp: torch.Tensor, params: dict, out=None,
                     d_index=None, stream=None):
    """lf_depth with the library's static device workspace (no caller workspace)."""
    vs = view_set(views)
    prm = make_params(params)
    _dev(hyp, torch.float32, "hyp")
    if out is None:
        out = torch.empty((vs.H, vs.W), dtype=torch.float32, device=views.device)
    _check(lib.lf_depth_noalloc(C.byref(vs), _ptr(hyp), hyp.shape[0], C.byref(prm), _ptr(out),
                                _ptr(d_index), _stream(stream)))
    return out


# ------------------------------------------------------------------ batches
def make_request(views: torch.Tensor, hyp: torch.Tensor, params: dict, disparity: torch.Tensor,
                 d_index=None) -> Request:
    _dev(hyp, torch.float32, "hyp")
    _dev(disparity, torch.float32, "disparity")
    if d_index is not None:
        _dev(d_index, torch.int16, "d_index")
    return Request(view_set(views), hyp.data_ptr(), hyp.shape[0], make_params(params),
                   disparity.data_ptr(), 0 if d_index is None else d_index.data_ptr())


def _requests(reqs):
    arr = (Request * len(reqs))(*reqs)
    return arr


def batch_workspace_bytes(reqs) -> int:
    arr = _requests(reqs)
    return lib.lf_batch_workspace_size(arr, len(reqs))


def make_tuning(t: dict | None) -> Tuning | None:
    if t is None:
        return None
    return Tuning(t.get("cost_cells_per_thread", 0), t.get("cost_stride", 0),
                  t.get("dense_prefetch", 0), t.get("bounded_prefetch", 0),
                  t.get("bounded_lanes", 0), t.get("bounded_offsets", 0))


class Plan:
    """A batch of light fields run together (lf_plan_*).  Keeps the request
    tensors and the workspace alive while the plan exists."""

    def __init__(self, items, ws=None, tuning: dict | None = None, stream=None):
        # items: sequence of (views, hyp, params, disparity, d_index or None)
        self._keep = list(items)
        reqs = [make_request(*it) for it in self._keep]
        self._arr = _requests(reqs)
        self.n = len(reqs)
        need = lib.lf_batch_workspace_size(self._arr, self.n)
        if need == 0:
            raise LFError(LF_EINVAL, "invalid batch")
        dev = self._keep[0][0].device
        self.ws = ws if ws is not None else workspace(need, dev)
        self._h = C.c_void_p()
        t = make_tuning(tuning)
        _check(lib.lf_plan_create(self._arr, self.n, _ptr(self.ws), self.ws.numel(),
                                  None if t is None else C.byref(t), _stream(stream),
                                  C.byref(self._h)))

    def autotune(self, reps: int = 2, stream=None) -> dict:
        t = Tuning()
        _check(lib.lf_plan_autotune(self._h, _stream(stream), reps, C.byref(t)))
        return t.as_dict()

    def capture(self):
        _check(lib.lf_plan_capture(self._h))

    def run(self, stream=None):
        _check(lib.lf_plan_run(self._h, _stream(stream)))

    @property
    def launches(self) -> int:
        return lib.lf_plan_launches(self._h)

    @property
    def tuning(self) -> dict:
        t = Tuning()
        _check(lib.lf_plan_tuning(self._h, C.byref(t)))
        return t.as_dict()

    def close(self):
        if self._h:
            lib.lf_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The request loop (lf_server_*) over a device arena of `arena_bytes`."""

    def __init__(self, arena_bytes: int, device, max_batch=16, max_inflight=2, max_queue=1024,
                 tuning: dict | None = None, arena=None, group_ratio=0, large_bytes=0,
                 max_large=0):
        self.arena = arena if arena is not None else workspace(arena_bytes, device)
        t = make_tuning(tuning) or Tuning()
        cfg = ServerConfig(self.arena.data_ptr(), self.arena.numel(), max_batch, max_inflight,
                           max_queue, group_ratio, t, large_bytes, max_large)
        self._h = C.c_void_p()
        _check(lib.lf_server_create(C.byref(cfg), C.byref(self._h)))
        self._keep = {}

    def submit(self, views, hyp, params, disparity, d_index=None, stream=None) -> int:
        """Queues a request; its work is ordered after what the current (or the
        given) torch stream has enqueued so far."""
        req = make_request(views, hyp, params, disparity, d_index)
        tk = C.c_int64()
        _check(lib.lf_server_submit(self._h, C.byref(req), _stream(stream), C.byref(tk)))
        self._keep[tk.value] = (views, hyp, disparity, d_index)
        return tk.value

    def wait(self, ticket: int, timeout: float = -1.0) -> dict:
        info = RequestInfo()
        st = lib.lf_server_wait(self._h, ticket, timeout, C.byref(info))
        if st == LF_ETIMEOUT:
            raise TimeoutError(f"ticket {ticket} still running")
        self._keep.pop(ticket, None)
        d = info.as_dict()
        if st != LF_OK:
            d["error"] = lib.lf_last_error().decode()
        return d

    def stats(self) -> dict:
        v = [C.c_int64() for _ in range(4)]
        lib.lf_server_stats(self._h, *[C.byref(x) for x in v])
        return dict(completed=v[0].value, batches=v[1].value, arena_in_use=v[2].value,
                    arena_peak=v[3].value)

    def close(self):
        if self._h:
            lib.lf_server_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
