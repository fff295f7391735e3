#!/usr/bin/env python3
"""Throughput of the light-field depth hot path on one MI355X.

A step is one whole pass of the method over one light field resident in HBM:
Census, initial Census cost + SGM + WTA over the cross views, fusion/fill/
borders, bounded l2 cost over all views, bounded SGM, WTA + sub-pixel + median
(lf_depth, i.e. the staged C-ABI calls back to back on one stream).

Workload: 9x9 views of 512x512 float32 in [0, 1], a seeded scene of 12 slanted
Perlin+noise planes, 100 hypotheses over [-4, 4], 7x9 Census, lambda = 3, 8 SGM
paths (synthetic stand-in for the 4D light field benchmark's shape).

Printed: one JSON line with Gcells/s (cells = |V|*H*W*N initial + the bounded
cells sum_p w(p)), depth maps/s, p50/p99 step latency, per-stage times from HIP
events recorded on the stream the kernels run on, the roofline of the dominant
kernel, and the CPU oracle timed on this host as a reported baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Gcells/s (pixel×hypothesis, cost+SGM) and depth maps/s at 9×9×512² "
          "vs plain; p99")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X fp32 vector


def stage_models(S, T, cells_initial, cells_bounded, sum_bits):
    """Algorithmic work of each stage per light field and the resource that bounds it.

    sgm_initial  (Census cost + SGM + WTA over the cross views): HBM, 12 B/cell --
                 the 16-bit aggregated cost must make 4 orientation round trips
                 (write, 3 x read+write, the last read fused into WTA).
    cost_bounded (l2 over all views, Eq. 12): fp32 ALU, 11 flop per view and cell
                 (3 FMA, 3 differences, |ref - val|, the running sum) over the
                 S*T - 1 views that are not the reference.
    sgm_bounded  (bounded SGM): HBM, 8 B/cell of cost reads (one per orientation)
                 plus 12 (16-bit sums) or 24 (32-bit sums) B/cell of sum state.
    """
    return {
        "sgm_initial": dict(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                            work=12.0 * cells_initial / 1e9,
                            kernel="census_cost_volume + sgm_dense_paths + dense_sum_wta"),
        "cost_bounded": dict(bound="alu", unit="TFLOP/s", peak=FP32_PEAK_TFLOPS,
                             work=11.0 * (S * T - 1) * cells_bounded / 1e12,
                             kernel="cost_l2_kernel"),
        "sgm_bounded": dict(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                            work=(8.0 + (12.0 if sum_bits == 16 else 24.0)) * cells_bounded / 1e9,
                            kernel="sgm_bounded_paths + bounded_sum"),
    }


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(kernel, src):
    """HBM bytes per launch of `kernel` measured by rocprofv3 counters (profiles/), or None
    if the counters were taken on another version of its source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}.traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    if rec.get("source_sha") != source_sha(src):
        return None
    try:
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(lfd, cells_per_map):
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.depth(lfd.views, lfd.hyp, lfd.params)
    dt = time.perf_counter() - t0
    return {"value": cells_per_map / dt / 1e9, "unit": "Gcells/s", "cores": 1,
            "kind": "oracle", "seconds_per_map": dt, "maps_per_s": 1.0 / dt,
            "sample": "one whole light field of the workload (9x9x512^2 f32, N=100), "
                      "single-threaded C oracle, -O3"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper", choices=["paper", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import lfsynth
    from paper_1907_13449_amd import lf

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    lfd = lfsynth.workload(args.workload)
    log(f"[bench] scene {lfd.name} generated in {time.perf_counter() - t0:.1f}s")
    views = torch.from_numpy(lfd.views).to(dev)
    hyp = torch.from_numpy(lfd.hyp).to(dev)
    p = lfd.params
    S, T, H, W, N = lfd.S, lfd.T, lfd.H, lfd.W, lfd.N
    ws = lf.workspace(lf.depth_workspace_bytes(S, T, H, W, N, p), dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    d_index = torch.empty((H, W), dtype=torch.int16, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        lf.lf_depth(views, hyp, p, ws=ws, out=out, d_index=d_index, stream=stream)

    # bounded cell count of this light field (from the staged calls' offsets)
    ini = lf.lf_initial_disparity(views, hyp, p)
    w = (ini["d_hi"].to(torch.int64) - ini["d_lo"].to(torch.int64) + 1)
    cells_bounded = int(w.sum().item())
    full_frac = float((w == N).float().mean().item())
    nv = len(lf.cross_views(S, T))
    cells_initial = nv * H * W * N
    cells = cells_initial + cells_bounded
    del ini, w

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done; timing {args.steps} steps")

    lf.profile_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    lf.profile_enable(False)
    stages = lf.profile_read()
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    gpu_ms = float(ev[0].elapsed_time(ev[-1]))
    ms_per_step = gpu_ms / args.steps
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall * 1e3 / args.steps:.3f})")

    stage_ms = {k: v[0] / args.steps for k, v in stages.items()}
    stage_launches = {k: v[1] // args.steps for k, v in stages.items()}
    models = stage_models(S, T, cells_initial, cells_bounded, p["sum_bits"])
    roofs = {}
    for name, m in models.items():
        sec = stage_ms[name] * 1e-3
        achieved = m["work"] / sec          # GB/s or TFLOP/s
        roofs[name] = {"kernel": m["kernel"], "bound": m["bound"], "achieved": achieved,
                       "peak": m["peak"], "unit": m["unit"], "frac": achieved / m["peak"],
                       "ms": stage_ms[name], "launches": stage_launches[name],
                       "avg_launch_ms": stage_ms[name] / max(stage_launches[name], 1)}
    dominant = max(roofs, key=lambda k: roofs[k]["ms"])
    src = {"sgm_initial": "sgm.hip", "sgm_bounded": "sgm.hip", "cost_bounded": "cost.hip"}
    roofline = dict(roofs[dominant])
    roofline["stage"] = dominant
    roofline["traffic"] = load_traffic(
        dominant, os.path.join(ROOT, "paper_1907_13449_amd", "csrc", src[dominant]))

    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    res = {
        "metric": METRIC,
        "value": cells * args.steps / (gpu_ms * 1e-3) / 1e9,
        "unit": "Gcells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u16",
        "data": "synthetic",
        "config": {"workload": f"{lfd.name}: {S}x{T} views of {H}x{W} "
                               f"{'u8' if lfd.views.dtype == np.uint8 else 'f32'}, N={N} over "
                               f"[{lfd.hyp[0]:.2f},{lfd.hyp[-1]:.2f}], Census "
                               f"{p['win_h']}x{p['win_w']}, lambda {p['lam']}, "
                               f"{p['npaths']} paths, plain per-light-field launch",
                   "cells_initial": cells_initial, "cells_bounded": cells_bounded,
                   "full_range_fraction": full_frac},
        "maps_per_s": 1000.0 / ms_per_step,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "stage_ms": stage_ms,
        "roofline": roofline,
        "stage_roofline": roofs,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on one light field")
        res["cpu_baseline"] = cpu_baseline(lfd, cells)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
