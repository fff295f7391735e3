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
unit (the initial stage's three kernels against the algorithmic bytes of that
stage), every stage's roofline and the whole step's fraction of HBM bandwidth,
with measured traffic from the committed rocprofv3 counter summaries when they
were taken on the current sources, and the CPU oracle timed on this host as a
reported baseline.

Also in the same line (skip them with --no-quality / --no-batch / --no-large /
--no-serve):
  quality  the map against the scene's ground truth (BadPix 0.07, MSE, M-metric of
           Sec. 4.2) beside the boundary-less search (lambda = -1, Sec. 4.5);
  batched  64 light fields mixing 5x5x256^2, 7x7x384^2 and 9x9x512^2 float32
           scenes with 32..128 hypotheses: one autotuned, graph-captured batch
           plan against the same 64 lf_depth calls one after another;
  batched_benchmark_shape  the same for 8 light fields of the benchmark shape
           (the benchmark scene plus seeded noise);
  large    2 x 15x15 views of 625x434 f32 (N = 64) with 2 x 1x11 views of
           1920x1080 u8 (N = 96): per shape and as one batch;
  served   Poisson arrivals (2,000 requests, 100 warm-up) drawn uniformly from the
           small 5x5x96^2 workload, the 9x9x512^2 N=100 workload and the mixed
           shapes above, through the request loop at 0.8 (and 0.5, 0.95) of the
           one-at-a-time capacity, against one-at-a-time lf_depth calls on the same
           arrival times: p50/p99 latency and maps/s.

Profile summaries (profiles/): --summarize-kernels and --summarize-counters turn
rocprofv3 output of this script into the committed tables and records.
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

# The paper's own runtime for this kind of light field (context, not a target):
# Table 1 / Sec. 4.7, a single thread of an Intel Xeon E3-1245 V2 at 3.40 GHz,
# 9x9 views of 512x512 8-bit RGB, 16 paths.
PAPER_RUNTIME = {"seconds_per_map_median": 10 ** 0.25, "seconds_per_map_average": 10 ** 0.23,
                 "hardware": "Intel Xeon E3-1245 V2 @ 3.40 GHz, one thread (C, GCC -O3)",
                 "workload": "4D light field benchmark: 9x9 views of 512x512 8-bit RGB, "
                             "16 SGM paths, sparse 7x7 Census",
                 "source": "Table 1 (Sec. 4.4), Sec. 4.7",
                 "note": "another machine, input and path count: context only"}

# Where each kernel's source lives (counter records are valid only for the source
# they were taken on) and which profiled stage launches it.
KERNEL_SOURCE = {
    "census_kernel": "census.hip", "census_cost_volume_kernel": "sgm.hip",
    "sgm_dense_paths_kernel": "sgm.hip", "dense_sum_wta_rows_kernel": "sgm.hip",
    "dense_sum_wta_kernel": "sgm.hip", "initial_export_kernel": "sgm.hip",
    "prep_kernel": "post.hip", "fuse_kernel": "post.hip", "fill_kernel": "post.hip",
    "borders_kernel": "post.hip", "full_range_kernel": "post.hip",
    "scan_reduce_kernel": "post.hip", "scan_apply_kernel": "post.hip",
    "pad_views_kernel": "cost.hip", "cost_l2_kernel": "cost.hip",
    "cost_census_all_kernel": "cost.hip", "pix_meta_kernel": "sgm.hip",
    "sgm_bounded_paths_kernel": "sgm.hip", "sgm_bounded_group_kernel": "sgm.hip",
    "bounded_sum_kernel": "sgm.hip", "wta_subpixel_kernel": "post.hip",
    "median3_kernel": "post.hip",
}
STAGE_KERNELS = {
    "census": ["census_kernel"],
    "sgm_initial": ["census_cost_volume_kernel", "sgm_dense_paths_kernel",
                    "dense_sum_wta_rows_kernel", "dense_sum_wta_kernel"],
    "fuse_fill_borders": ["prep_kernel", "fuse_kernel", "fill_kernel", "borders_kernel"],
    "offsets": ["scan_reduce_kernel", "scan_apply_kernel"],
    "cost_inputs": ["pad_views_kernel"],
    "cost_bounded": ["cost_l2_kernel", "cost_census_all_kernel"],
    "sgm_bounded": ["pix_meta_kernel", "sgm_bounded_paths_kernel", "sgm_bounded_group_kernel",
                    "bounded_sum_kernel"],
    "wta_subpixel_median": ["wta_subpixel_kernel", "median3_kernel"],
}


def algorithmic_work(S, T, H, W, N, nv, px_bytes, cells_initial, cells_bounded, sum_bits):
    """Algorithmic work of every stage of one light field and the resource that bounds
    it, from the data each step must move (not what this design moves):

    census               (pixel bytes + 8) per pixel of the reference and cross views
    sgm_initial          12 B per initial cell -- the 16-bit aggregated cost makes its
                         round trips between the four orientation passes (written once,
                         read and written twice, read once by the WTA) -- plus
                         (2*8 + 2)/N B per cell for the two Census strings and D_i
    fuse_fill_borders    ~40 B per pixel (maps, d_init, bounds), offsets included
    cost_inputs          0 (the edge-replicated view copy is this design's choice)
    cost_bounded         fp32 ALU: 11 flop per view and cell (3 FMA, 3 differences,
                         |ref - val|, the running sum) over the S*T - 1 views that are
                         not the reference; bytes: the 16-bit cost written and every
                         view read once
    sgm_bounded          8 B per cell of cost reads (one per orientation) + 12 (16-bit
                         sums) or 24 (32-bit sums) B per cell of aggregated-cost state
    wta_subpixel_median  ~12 B per pixel
    """
    HW = H * W
    work = {
        "census": dict(bytes=(px_bytes + 8) * HW * (1 + nv)),
        "sgm_initial": dict(bytes=(12.0 + 18.0 / N) * cells_initial),
        "fuse_fill_borders": dict(bytes=40.0 * HW),
        "offsets": dict(bytes=0.0),
        "cost_inputs": dict(bytes=0.0),
        "cost_bounded": dict(bytes=2.0 * cells_bounded + (S * T * px_bytes + 8.0) * HW,
                             flop=11.0 * (S * T - 1) * cells_bounded),
        "sgm_bounded": dict(bytes=(8.0 + (12.0 if sum_bits == 16 else 24.0)) * cells_bounded),
        "wta_subpixel_median": dict(bytes=12.0 * HW),
    }
    return work


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


CSRC = os.path.join(ROOT, "paper_1907_13449_amd", "csrc")


def current_sources():
    """sha256 (16 hex) of every kernel source and the shared internal header."""
    names = sorted(set(KERNEL_SOURCE.values())) + ["lf_internal.h"]
    return {n: source_sha(os.path.join(CSRC, n)) for n in names}


def load_counter_record(workload_name):
    """Per-kernel HBM traffic (rocprofv3 FETCH_SIZE / WRITE_SIZE, calibrated) of the
    workload from profiles/traffic_<workload>.json, keeping only the kernels whose
    source (and the shared header) is the one the counters were taken on."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_name}.json")
    if not os.path.exists(path):
        return {}
    rec = json.load(open(path))
    cur = current_sources()
    srcs = rec.get("sources", {})
    ok = {}
    for k, v in rec.get("kernels", {}).items():
        src = KERNEL_SOURCE.get(k)
        if src and srcs.get(src) == cur.get(src) and srcs.get("lf_internal.h") == cur.get(
                "lf_internal.h"):
            ok[k] = v
    return ok


def cpu_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def time_oracle(lfd, runs):
    """Seconds per whole light field of the oracle, over `runs` runs, this thread
    pinned to one core (the affinity is restored afterwards)."""
    import oracle
    oracle.build(force=False)
    before = os.sched_getaffinity(0)
    core = min(before)
    os.sched_setaffinity(0, {core})
    try:
        times = []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.depth(lfd.views, lfd.hyp, lfd.params)
            times.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, before)
    return times, core


def cpu_baseline(lfd, cells_per_map, small=None, small_cells=None, runs=3):
    """The oracle (single-threaded C, -O3) on whole light fields of the benchmark
    workload, `runs` runs pinned to one core, plus five runs of the small workload."""
    times, core = time_oracle(lfd, runs)
    dt = sum(times) / len(times)
    res = {"value": cells_per_map / dt / 1e9, "unit": "Gcells/s", "cores": 1, "kind": "oracle",
           "seconds_per_map": dt, "seconds_per_map_runs": times, "maps_per_s": 1.0 / dt,
           "runs": runs, "pinned_core": core, **cpu_info(),
           "sample": f"{runs} runs of the oracle on one whole light field of the workload "
                     f"({lfd.S}x{lfd.T} views of {lfd.H}x{lfd.W}, N={lfd.N}; "
                     f"{sum(times):.1f} s of CPU work), one thread pinned to one core"}
    if small is not None:
        st, _ = time_oracle(small, 5)
        sd = sum(st) / len(st)
        res["small"] = {"workload": f"{small.S}x{small.T} views of {small.H}x{small.W} u8, "
                                    f"N={small.N}", "seconds_per_map": sd,
                        "gcells_s": small_cells / sd / 1e9 if small_cells else None, "runs": 5}
    return res


# ----------------------------------------------------- rocprofv3 summaries
def _short_kernel(name):
    """'void lf::(anonymous namespace)::foo_kernel<lf::Single<...>, ...>(...)' ->
    ('foo_kernel', 'Single')."""
    import re
    m = re.search(r"::(\w+_kernel)<lf::(Single|Group)<", name)
    if m:
        return m.group(1), m.group(2)
    return name.split("(")[0].split("<")[0].split("::")[-1], ""


def summarize_kernel_stats(stats_csv, command):
    """Markdown of a rocprofv3 --kernel-trace --stats summary: calls and average
    microseconds per kernel (liblf kernels by short name and launch form)."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    out = [f"Command (from the repository root, on one MI355X):", "", f"    {command}", "",
           "Sources: " + ", ".join(f"{k} {v}" for k, v in current_sources().items()) +
           " (sha256, 16 hex).", "",
           "| kernel | form | calls | avg us | total % |", "|---|---|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        k, form = _short_kernel(r["Name"])
        out.append(f"| {k} | {form} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out)


def summarize_counters(fetch_csv, write_csv, calib_bytes, workload_name, commands):
    """Per-kernel HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE and
    WRITE_SIZE, KiB per dispatch).  Each counter is scaled by what it reads for the
    plain device copy of calib_bytes in the same run (the largest non-liblf dispatch):
    fetched bytes = FETCH_SIZE x calib_bytes / FETCH_SIZE(copy), likewise written.
    Returns (record dict, markdown)."""
    import csv
    import statistics

    def per_dispatch(path, counter):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") != counter:
                continue
            key = (r["Dispatch_Id"], r["Kernel_Name"])
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
        return vals

    f, w = per_dispatch(fetch_csv, "FETCH_SIZE"), per_dispatch(write_csv, "WRITE_SIZE")

    def calib(vals):
        other = [v for (d, n), v in vals.items() if "lf::" not in n]
        return calib_bytes / (max(other) * 1024.0)

    ff, wf = calib(f), calib(w)

    def by_kernel(vals, factor):
        acc = {}
        for (d, n), v in vals.items():
            if "lf::" not in n:
                continue
            k, form = _short_kernel(n)
            acc.setdefault(k, []).append(v * 1024.0 * factor)
        return {k: (statistics.median(v), len(v)) for k, v in acc.items()}

    fk, wk = by_kernel(f, ff), by_kernel(w, wf)
    kernels = {}
    for k in sorted(set(fk) | set(wk)):
        kernels[k] = {"fetch_bytes": fk.get(k, (0.0, 0))[0], "write_bytes": wk.get(k, (0.0, 0))[0],
                      "launches": max(fk.get(k, (0, 0))[1], wk.get(k, (0, 0))[1])}
    rec = {"workload": workload_name, "commands": commands, "calib_bytes": calib_bytes,
           "fetch_factor": ff, "write_factor": wf, "sources": current_sources(),
           "kernels": kernels}
    md = [f"Commands (from the repository root, one counter per run, on one MI355X):", ""]
    md += [f"    {c}" for c in commands]
    md += ["", f"Calibration: the plain {calib_bytes / 2**30:.0f} GiB device copy in the same run "
           f"reads FETCH_SIZE x {ff:.3f} KiB and WRITE_SIZE x {wf:.3f} KiB per byte moved, "
           "so fetched bytes = FETCH_SIZE x 1024 x that factor, likewise written.", "",
           "Per launch (median over the run's dispatches of each kernel):", "",
           "| kernel | launches | fetched MB | written MB |", "|---|---:|---:|---:|"]
    for k, v in sorted(kernels.items(), key=lambda x: -(x[1]["fetch_bytes"] + x[1]["write_bytes"])):
        md.append(f"| {k} | {v['launches']} | {v['fetch_bytes'] / 1e6:.1f} | "
                  f"{v['write_bytes'] / 1e6:.1f} |")
    return rec, "\n".join(md)


# --------------------------------------------------------------- quality
def quality_vs_boundless(lf, lfd, views, hyp, out, ms_bounded, cells_bounded, stream, steps=5):
    """Sec. 4.2 measures of the headline map against the scene's ground truth, beside
    the boundary-less search (Sec. 4.5: lambda = -1, every pixel over the full
    range, no initial map) on the same light field: what the bounds save in cells
    and time, and what they cost or gain in accuracy."""
    import numpy as np
    import torch
    from paper_1907_13449_amd import quality
    # pixels whose largest shift can reach past the image edge are left out
    dmax = float(max(abs(lfd.hyp[0]), abs(lfd.hyp[-1])))
    border = int(np.ceil(dmax * (max(lfd.S, lfd.T) - 1) / 2))
    H, W, N = lfd.H, lfd.W, lfd.N
    torch.cuda.synchronize()
    bounded = out.cpu().numpy()
    p = dict(lfd.params, lam=-1)
    ws = lf.workspace(lf.depth_workspace_bytes(lfd.S, lfd.T, H, W, N, p), views.device)
    free = torch.empty_like(out)
    lf.lf_depth(views, hyp, p, ws=ws, out=free, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        lf.lf_depth(views, hyp, p, ws=ws, out=free, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_free = e0.elapsed_time(e1) / steps
    free_map = free.cpu().numpy()
    del ws

    def q(m, ms):
        bp = quality.badpix(m, lfd.gt, 0.07, border)
        return {"badpix_0.07": bp, "mse": quality.mse(m, lfd.gt, border), "ms": ms,
                "m_metric_pct_per_s": quality.m_metric(bp, ms * 1e-3)}
    res = {"border_px": border, "ground_truth": "synthetic scene disparity (reference view)",
           "bounded": dict(q(bounded, ms_bounded), final_cells=cells_bounded),
           "boundless": dict(q(free_map, ms_free), final_cells=H * W * N),
           "hypotheses_saved": 1.0 - cells_bounded / (H * W * N),
           "time_saved": 1.0 - ms_bounded / ms_free}
    log(f"[bench] bounded: BadPix {res['bounded']['badpix_0.07']:.2f} % in {ms_bounded:.2f} ms; "
        f"boundary-less: BadPix {res['boundless']['badpix_0.07']:.2f} % in {ms_free:.2f} ms")

    # one reading or parameter of the bounded method changed at a time: what each
    # costs or buys in accuracy, cells and time on this scene
    variants = {"lambda_6": dict(lam=6), "lambda_10": dict(lam=10), "lambda_20": dict(lam=20),
                "no_edge_exclusion": dict(edge_tau=float("inf")), "no_fill": dict(fill_passes=0),
                "phi_1": dict(phi=1), "phi_8": dict(phi=8), "adaptive_lambda_far_8": dict(lam_far=8)}
    abl = {}
    for name, change in variants.items():
        pv = dict(lfd.params, **change)
        ws = lf.workspace(lf.depth_workspace_bytes(lfd.S, lfd.T, H, W, N, pv), views.device)
        m = torch.empty_like(out)
        lf.lf_depth(views, hyp, pv, ws=ws, out=m, stream=stream)
        e0.record(stream)
        for _ in range(steps):
            lf.lf_depth(views, hyp, pv, ws=ws, out=m, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ini = lf.lf_initial_disparity(views, hyp, pv, want_maps=False)
        w = (ini["d_hi"].to(torch.int64) - ini["d_lo"].to(torch.int64) + 1)
        shown = {k: (v if np.isfinite(v) else str(v)) for k, v in change.items()}   # JSON
        abl[name] = dict(q(m.cpu().numpy(), ms), change=shown, final_cells=int(w.sum().item()),
                         full_range_fraction=float((w == N).float().mean().item()))
        del ws, ini, w
    res["ablation"] = abl
    log("[bench] ablation: " + ", ".join(f"{k} {v['badpix_0.07']:.2f} % / {v['ms']:.2f} ms"
                                          for k, v in abl.items()))
    return res


def summarize_units(sq_csv, ta_csv, td_csv, commands):
    """Markdown of per-kernel unit utilisation from three rocprofv3 --pmc runs:
    SQ instruction and wave counters; TA_TA_BUSY_sum with GRBM_GUI_ACTIVE; TD_TD_BUSY_sum
    with GRBM_GUI_ACTIVE.  The median over each kernel's dispatches; GRBM_GUI_ACTIVE
    sums the 8 XCDs, so kernel cycles = GRBM_GUI_ACTIVE / 8; VALU busy = SQ_INSTS_VALU
    x 4 cycles (a wave64 instruction on a 16-lane SIMD) / (1,024 SIMDs x cycles);
    TA / TD busy = TA_TA_BUSY_sum / TD_TD_BUSY_sum / (256 CUs x cycles)."""
    import csv
    import statistics

    def per_kernel(path):
        vals = {}
        for r in csv.DictReader(open(path)):
            if "lf::" not in r["Kernel_Name"]:
                continue
            key = (r["Dispatch_Id"], r["Kernel_Name"], r["Counter_Name"])
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
        acc = {}
        for (d, n, c), v in vals.items():
            acc.setdefault(_short_kernel(n)[0], {}).setdefault(c, []).append(v)
        return {k: {c: statistics.median(v) for c, v in cs.items()} for k, cs in acc.items()}

    sq, ta, td = per_kernel(sq_csv), per_kernel(ta_csv), per_kernel(td_csv)
    rows = []
    for k in sq:
        cyc_ta = ta.get(k, {}).get("GRBM_GUI_ACTIVE", 0.0) / 8.0
        cyc_td = td.get(k, {}).get("GRBM_GUI_ACTIVE", 0.0) / 8.0
        if cyc_ta <= 0 or cyc_td <= 0:
            continue
        valu = sq[k].get("SQ_INSTS_VALU", 0.0)
        rows.append((cyc_ta / 2.4e3, k, 100.0 * valu * 4 / (1024 * cyc_ta),
                     100.0 * ta[k].get("TA_TA_BUSY_sum", 0.0) / (256 * cyc_ta),
                     100.0 * td[k].get("TD_TD_BUSY_sum", 0.0) / (256 * cyc_td),
                     sq[k].get("SQ_INSTS_VMEM_RD", 0.0) / 1e6, sq[k].get("SQ_INSTS_VMEM_WR", 0.0) / 1e6,
                     valu / 1e6, sq[k].get("SQ_INSTS_SALU", 0.0) / 1e6))
    md = ["Commands (from the repository root, one counter set per run, on one MI355X):", ""]
    md += [f"    {c}" for c in commands]
    md += ["", "Sources: " + ", ".join(f"{k} {v}" for k, v in current_sources().items()) +
           " (sha256, 16 hex).", "",
           "Normalisation (median over each kernel's dispatches): kernel cycles = "
           "GRBM_GUI_ACTIVE / 8 (the counter sums the 8 XCDs); VALU busy = SQ_INSTS_VALU x 4 "
           "cycles (a wave64 instruction on a 16-lane SIMD) / (1,024 SIMDs x kernel cycles); "
           "TA / TD busy = TA_TA_BUSY_sum / TD_TD_BUSY_sum / (256 CUs x kernel cycles).  Time "
           "is kernel cycles at 2.4 GHz under the profiler.", "",
           "| kernel | us | VALU busy % | TA busy % | TD busy % | vector loads (M wave instr) "
           "| vector stores (M) | VALU (M wave instr) | SALU (M) |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in sorted(rows, reverse=True):
        md.append(f"| {r[1]} | {r[0]:.0f} | {r[2]:.0f} | {r[3]:.0f} | {r[4]:.0f} | {r[5]:.2f} | "
                  f"{r[6]:.2f} | {r[7]:.1f} | {r[8]:.1f} |")
    return "\n".join(md)


def summarize_stalls(sq_csv, commands):
    """Markdown of where each kernel's waves spend their cycles, from one rocprofv3
    --pmc run of SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU
    SQ_ACTIVE_INST_VMEM SQ_INST_LEVEL_VMEM SQ_VMEM_TA_ADDR_FIFO_FULL
    SQ_VMEM_TA_CMD_FIFO_FULL (medians over each kernel's dispatches).  Each wave
    counter is divided by SQ_WAVE_CYCLES: SQ_WAIT_ANY counts wave cycles spent in
    s_waitcnt (waiting for memory), SQ_WAIT_INST_ANY wave cycles with an
    instruction ready but not issued (its unit or the issue slot taken by another
    wave), SQ_ACTIVE_INST_* wave cycles issuing that kind, and SQ_INST_LEVEL_VMEM /
    SQ_WAVE_CYCLES a relative measure of its vector-memory instructions in flight."""
    import csv
    import statistics
    vals = {}
    for r in csv.DictReader(open(sq_csv)):
        if "lf::" not in r["Kernel_Name"]:
            continue
        key = (r["Dispatch_Id"], r["Kernel_Name"], r["Counter_Name"])
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    acc = {}
    for (d, n, c), v in vals.items():
        acc.setdefault(_short_kernel(n)[0], {}).setdefault(c, []).append(v)
    med = {k: {c: statistics.median(v) for c, v in cs.items()} for k, cs in acc.items()}
    rows = []
    for k, m in med.items():
        wc = m.get("SQ_WAVE_CYCLES", 0.0)
        if wc <= 0:
            continue
        rows.append((wc, k, *(m.get(c, 0.0) / wc for c in (
            "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_VMEM",
            "SQ_INST_LEVEL_VMEM")),
            m.get("SQ_VMEM_TA_ADDR_FIFO_FULL", 0.0) + m.get("SQ_VMEM_TA_CMD_FIFO_FULL", 0.0)))
    md = ["Command (from the repository root, on one MI355X):", ""]
    md += [f"    {c}" for c in commands]
    md += ["", "Sources: " + ", ".join(f"{k} {v}" for k, v in current_sources().items()) +
           " (sha256, 16 hex).", "",
           "Fractions of the kernel's wave cycles (medians over its dispatches): waiting in "
           "s_waitcnt (SQ_WAIT_ANY), ready but not issued (SQ_WAIT_INST_ANY), issuing VALU / "
           "vector-memory instructions (SQ_ACTIVE_INST_VALU / _VMEM); SQ_INST_LEVEL_VMEM / SQ_WAVE_CYCLES, a "
           "relative measure of vector-memory instructions in flight (for comparing kernels); "
           "cycles the texture address unit's FIFOs were full (ADDR + CMD).", "",
           "| kernel | wave cycles (M) | s_waitcnt | not issued | VALU | VMEM | VMEM level "
           "| TA FIFO full |", "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for r in sorted(rows, reverse=True):
        md.append(f"| {r[1]} | {r[0] / 1e6:.1f} | {r[2]:.2f} | {r[3]:.2f} | {r[4]:.2f} | "
                  f"{r[5]:.2f} | {r[6]:.2f} | {r[7]:.3g} |")
    return "\n".join(md)


def summarize_plan_gaps(trace_csv, command):
    """Markdown of a rocprofv3 --kernel-trace of --replay-plan: per replay of the
    captured plan, its liblf kernels, the span from the first start to the last
    end, and the time within it when none of them ran."""
    import csv
    rows = [r for r in csv.DictReader(open(trace_csv)) if "lf::" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    runs, cur = [], [rows[0]]
    for a, b in zip(rows, rows[1:]):       # replays are separated by host sleeps
        if int(b["Start_Timestamp"]) - int(a["End_Timestamp"]) > 5_000_000:
            runs.append(cur)
            cur = []
        cur.append(b)
    runs.append(cur)
    md = ["Command (from the repository root, on one MI355X):", "", f"    {command}", "",
          "Sources: " + ", ".join(f"{k} {v}" for k, v in current_sources().items()) +
          " (sha256, 16 hex).", "",
          "| replay | kernels | span ms | kernels running ms | idle ms |", "|---:|---:|---:|---:|---:|"]
    for i, run in enumerate(runs):
        t0 = int(run[0]["Start_Timestamp"])
        t1 = max(int(r["End_Timestamp"]) for r in run)
        busy, last = 0, t0
        for r in run:
            s, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            if e > last:
                busy += e - max(s, last)
                last = e
        md.append(f"| {i} | {len(run)} | {(t1 - t0) / 1e6:.3f} | {busy / 1e6:.3f} | "
                  f"{(t1 - t0 - busy) / 1e6:.3f} |")
    return "\n".join(md)


def replay_plan(dev, n=64, replays=3):
    """The batched workload's plan (fixed tuning), captured and replayed `replays`
    times with a host sleep between replays (for a kernel trace of the replays)."""
    import torch
    import lfsynth
    from paper_1907_13449_amd import lf
    scenes = mixed_scenes(lfsynth.workload("paper"), dev)
    reqs = mixed_requests(scenes, n, 3, dev, cycle=True)
    outs = [torch.empty(r["views"].shape[2:], dtype=torch.float32, device=dev) for r in reqs]
    plan = lf.Plan([(r["views"], r["hyp"], r["params"], o, None) for r, o in zip(reqs, outs)],
                   tuning=dict(cost_cells_per_thread=4, cost_stride=1, dense_prefetch=16,
                               bounded_prefetch=16, bounded_lanes=32))
    plan.capture()
    stream = torch.cuda.current_stream()
    for _ in range(2):
        plan.run(stream)
    torch.cuda.synchronize()
    for _ in range(replays):
        time.sleep(0.02)
        plan.run(stream)
        torch.cuda.synchronize()
    log(f"[bench] replayed the {n}-light-field plan {replays} times ({plan.launches} launches)")
    plan.close()


# --------------------------------------------------------------- batches
def mixed_scenes(paper_lfd, dev):
    """Device-resident scenes of the batched and served workloads: the 9x9x512^2
    scene of the headline workload, one seeded 5x5x256^2 and one 7x7x384^2 scene
    of the same family (slanted Perlin+noise planes, disparity in [-4, 4]), and
    the small 5x5x96^2 uint8 workload."""
    import torch
    import lfsynth
    t0 = time.perf_counter()
    out = {}
    for key, (S, H) in {"5x5x256": (5, 256), "7x7x384": (7, 384)}.items():
        l = lfsynth.workload("paper_s", seed=20 + S, H=H, W=H, S=S, T=S, N=64)
        out[key] = (torch.from_numpy(l.views).to(dev), l.params)
    out["9x9x512"] = (torch.from_numpy(paper_lfd.views).to(dev), paper_lfd.params)
    small = lfsynth.workload("small")
    out["small"] = (torch.from_numpy(small.views).to(dev), small.params,
                    torch.from_numpy(small.hyp).to(dev))
    log(f"[bench] mixed scenes generated in {time.perf_counter() - t0:.1f}s")
    return out


def mixed_requests(scenes, n, seed, dev, kinds=("5x5x256", "7x7x384", "9x9x512"), cycle=False):
    """n requests over `kinds` (in turn if `cycle`, else drawn uniformly); each of the
    three f32 shapes gets N drawn from 32..128 over [-4, 4], "mix" is one of those
    three drawn uniformly, "paper" is the 9x9x512^2 workload with N = 100, and
    "small" keeps its own N = 32 over [-2, 2] and parameters."""
    import numpy as np
    import torch
    import lfsynth
    shapes = ("5x5x256", "7x7x384", "9x9x512")
    rng = np.random.default_rng(seed)
    reqs = []
    hyps = {}
    for i in range(n):
        kind = kinds[i % len(kinds)] if cycle else kinds[int(rng.integers(len(kinds)))]
        if kind == "mix":
            kind = shapes[int(rng.integers(3))]
        if kind == "small":
            views, params, hyp = scenes["small"]
        elif kind == "paper":                   # the 9x9x512^2 workload, N = 100
            views, params = scenes["9x9x512"]
            if 100 not in hyps:
                hyps[100] = torch.from_numpy(lfsynth.hypotheses(-4.0, 4.0, 100)).to(dev)
            hyp = hyps[100]
        else:
            views, params = scenes[kind]
            N = int(rng.integers(32, 129))
            if N not in hyps:
                hyps[N] = torch.from_numpy(lfsynth.hypotheses(-4.0, 4.0, N)).to(dev)
            hyp = hyps[N]
        reqs.append(dict(kind=kind, views=views, hyp=hyp, params=params))
    return reqs


def request_cells(lf, r):
    """Cells of one request: |V|*H*W*N initial + the bounded cells of its ranges."""
    import torch
    ini = lf.lf_initial_disparity(r["views"], r["hyp"], r["params"], want_maps=False)
    w = ini["d_hi"].to(torch.int64) - ini["d_lo"].to(torch.int64) + 1
    T, S, H, W = r["views"].shape
    return len(lf.cross_views(S, T)) * H * W * r["hyp"].shape[0] + int(w.sum().item())


def run_batched(scenes, n, dev):
    reqs = mixed_requests(scenes, n, 3, dev, cycle=True)
    return time_batch(reqs, dev, f"{n} light fields: 5x5x256^2 / 7x7x384^2 / 9x9x512^2 f32, "
                                 "N in 32..128")


def run_batched_benchmark_shape(views, hyp, params, n, dev):
    """n light fields of the benchmark shape (9x9x512^2 f32, N = 100) as one batch
    against n lf_depth calls: the benchmark light field plus seeded Gaussian noise
    (sigma 0.004) drawn on the GPU, so that no two members are equal."""
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(2024)
    reqs = []
    for i in range(n):
        v = (views + 0.004 * torch.randn(views.shape, generator=g, device=dev)).clamp_(0.0, 1.0)
        reqs.append(dict(kind="paper", views=v, hyp=hyp, params=params))
    return time_batch(reqs, dev, f"{n} light fields of 9x9x512^2 f32, N = 100 "
                                 "(the benchmark scene with seeded noise)")


def time_batch(reqs, dev, label):
    """Plain (one lf_depth per light field, back to back on one stream) against one
    autotuned, graph-captured plan over the same light fields."""
    import numpy as np
    import torch
    from paper_1907_13449_amd import lf
    n = len(reqs)
    cells = sum(request_cells(lf, r) for r in reqs)
    outs = [torch.empty(r["views"].shape[2:], dtype=torch.float32, device=dev) for r in reqs]
    # plain: one lf_depth per light field, back to back on one stream, one workspace
    need = max(lf.depth_workspace_bytes(r["views"].shape[1], r["views"].shape[0],
                                        r["views"].shape[2], r["views"].shape[3],
                                        r["hyp"].shape[0], r["params"]) for r in reqs)
    ws = lf.workspace(need, dev)
    stream = torch.cuda.current_stream()

    def plain():
        for r, o in zip(reqs, outs):
            lf.lf_depth(r["views"], r["hyp"], r["params"], ws=ws, out=o, stream=stream)

    plain()
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plain()
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / reps
    del ws
    # batched: one plan, autotuned on its own inputs, captured, replayed
    t0 = time.perf_counter()
    plan = lf.Plan([(r["views"], r["hyp"], r["params"], o, None) for r, o in zip(reqs, outs)])
    tuning = plan.autotune(reps=1)
    plan.capture()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    for o in outs:
        o.fill_(float("nan"))
    plan.run(stream)
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(outs, ref))
    e0.record(stream)
    for _ in range(reps):
        plan.run(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1) / reps
    res = {"workload": label,
           "light_fields": n, "cells": cells,
           "batched_ms": batch_ms, "plain_ms": plain_ms,
           "batched_gcells_s": cells / (batch_ms * 1e-3) / 1e9,
           "plain_gcells_s": cells / (plain_ms * 1e-3) / 1e9,
           "batched_maps_s": n / (batch_ms * 1e-3), "plain_maps_s": n / (plain_ms * 1e-3),
           "speedup": plain_ms / batch_ms, "identical_to_plain": bool(same),
           "launches_per_batch": plan.launches, "tuning": tuning,
           "plan_setup_s": setup_s, "graph": True}
    plan.close()
    log(f"[bench] batched {label}: {batch_ms:.2f} ms vs plain {plain_ms:.2f} ms "
        f"({plain_ms / batch_ms:.2f}x), identical={same}")
    return res


def run_large(dev, reps=3):
    """The large workload: two 15x15-view plenoptic-like light fields of 625x434 f32
    (N = 64, d in [-1.5, 1.5], noise 0.01; seeds 4001, 4002) and two 1x11
    moving-stage light fields of 1920x1080 u8 (N = 96, d in [0, 24]; seeds 4003,
    4004), 8 paths.  Plain: one lf_depth per light field back to back, with
    per-stage times of each shape from the library's event hook; batched: the four
    as one autotuned, graph-captured plan."""
    import numpy as np
    import torch
    import lfsynth
    from paper_1907_13449_amd import lf
    t0 = time.perf_counter()
    lfds = [lfsynth.workload("plenoptic", seed=4001), lfsynth.workload("plenoptic", seed=4002),
            lfsynth.workload("stage", seed=4003), lfsynth.workload("stage", seed=4004)]
    log(f"[bench] large workload generated in {time.perf_counter() - t0:.1f}s")
    reqs = [dict(kind="plenoptic" if l.S == 15 else "stage", lfd=l,
                 views=torch.from_numpy(l.views).to(dev), hyp=torch.from_numpy(l.hyp).to(dev),
                 params=l.params) for l in lfds]
    cells = [request_cells(lf, r) for r in reqs]
    outs = [torch.empty((r["lfd"].H, r["lfd"].W), dtype=torch.float32, device=dev) for r in reqs]
    need = max(lf.depth_workspace_bytes(r["lfd"].S, r["lfd"].T, r["lfd"].H, r["lfd"].W,
                                        r["lfd"].N, r["params"]) for r in reqs)
    ws = lf.workspace(need, dev)
    stream = torch.cuda.current_stream()

    def one(r, o):
        lf.lf_depth(r["views"], r["hyp"], r["params"], ws=ws, out=o, stream=stream)

    for r, o in zip(reqs, outs):
        one(r, o)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    # per light field: time and stages (hook on), then the whole sequence (hook off)
    per = {}
    for r, o, c in zip(reqs, outs, cells):
        lf.profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            one(r, o)
        e1.record(stream)
        torch.cuda.synchronize()
        lf.profile_enable(False)
        st = lf.profile_read()
        d = per.setdefault(r["kind"], {"ms": [], "cells": [], "stage_ms": {}})
        d["ms"].append(e0.elapsed_time(e1) / reps)
        d["cells"].append(c)
        for k, v in st.items():
            d["stage_ms"][k] = d["stage_ms"].get(k, 0.0) + v[0] / reps / 2.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        for r, o in zip(reqs, outs):
            one(r, o)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / reps
    del ws
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    plan = lf.Plan([(r["views"], r["hyp"], r["params"], o, None) for r, o in zip(reqs, outs)])
    tuning = plan.autotune(reps=1)
    plan.capture()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    for o in outs:
        o.fill_(float("nan"))
    plan.run(stream)
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(outs, ref))
    e0.record(stream)
    for _ in range(reps):
        plan.run(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1) / reps
    plan.close()
    total = float(sum(cells))
    shapes = {}
    for kind, d in per.items():
        l = next(r["lfd"] for r in reqs if r["kind"] == kind)
        ms = float(np.mean(d["ms"]))
        shapes[kind] = {"shape": f"{l.S}x{l.T} views of {l.W}x{l.H} "
                                 f"{'u8' if l.views.dtype == np.uint8 else 'f32'}, N={l.N}, "
                                 f"d in [{l.hyp[0]:.1f}, {l.hyp[-1]:.1f}]",
                        "ms_per_map": ms, "cells_per_map": float(np.mean(d["cells"])),
                        "gcells_s": float(np.mean(d["cells"])) / (ms * 1e-3) / 1e9,
                        "stage_ms": {k: v for k, v in d["stage_ms"].items() if v > 0}}
    res = {"workload": "2 x 15x15x625x434 f32 (N=64) + 2 x 1x11x1920x1080 u8 (N=96), 8 paths",
           "light_fields": len(reqs), "cells": total, "plain_ms": plain_ms, "batched_ms": batch_ms,
           "plain_gcells_s": total / (plain_ms * 1e-3) / 1e9,
           "batched_gcells_s": total / (batch_ms * 1e-3) / 1e9,
           "plain_maps_s": len(reqs) / (plain_ms * 1e-3),
           "batched_maps_s": len(reqs) / (batch_ms * 1e-3), "speedup": plain_ms / batch_ms,
           "identical_to_plain": bool(same), "tuning": tuning, "plan_setup_s": setup_s,
           "per_shape": shapes}
    log(f"[bench] large: batched {batch_ms:.2f} ms vs plain {plain_ms:.2f} ms "
        f"({plain_ms / batch_ms:.2f}x), {res['plain_gcells_s']:.1f} Gcells/s plain")
    return res


def run_served(scenes, n, warmup, dev, rates=(0.8, 0.5, 0.95)):
    """Poisson arrivals of requests drawn uniformly from the small 5x5x96^2 u8
    workload, the 9x9x512^2 N=100 workload and the mixed shapes (5x5x256^2,
    7x7x384^2, 9x9x512^2 f32, N in 32..128), each at a fixed rate rho x the
    one-at-a-time capacity measured from the requests' own service times: rho = 0.8
    reported, 0.5 and 0.95 as a sweep.  n requests, the first `warmup` of them not
    counted.  Plain = a FIFO loop of lf_depth calls, each started at or after its
    arrival; served = the request loop over a resident arena, on the same arrivals.
    Latency = completion - arrival."""
    import numpy as np
    import torch
    from paper_1907_13449_amd import lf
    reqs = mixed_requests(scenes, n, 11, dev, kinds=("small", "paper", "mix"))
    outs = [torch.empty(r["views"].shape[2:], dtype=torch.float32, device=dev) for r in reqs]
    need = max(lf.depth_workspace_bytes(r["views"].shape[1], r["views"].shape[0],
                                        r["views"].shape[2], r["views"].shape[3],
                                        r["hyp"].shape[0], r["params"]) for r in reqs)
    ws = lf.workspace(need, dev)
    stream = torch.cuda.current_stream()
    for r, o in zip(reqs, outs):
        lf.lf_depth(r["views"], r["hyp"], r["params"], ws=ws, out=o, stream=stream)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    # service time of each request alone (plain launch), for the arrival rate
    svc = []
    for r, o in zip(reqs, outs):
        t = time.perf_counter()
        lf.lf_depth(r["views"], r["hyp"], r["params"], ws=ws, out=o, stream=stream)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t)
    mean_svc = float(np.mean(svc))
    counted = slice(warmup, n)

    def pct(lat):
        lat = np.asarray(lat)[counted]
        return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3)}

    def wait_until(t0, a):
        while time.perf_counter() - t0 < a:
            pass

    def plain(arr):
        t0 = time.perf_counter()
        lat, done, first = [], 0.0, None
        for i, (r, o, a) in enumerate(zip(reqs, outs, arr)):
            wait_until(t0, a)
            lf.lf_depth(r["views"], r["hyp"], r["params"], ws=ws, out=o, stream=stream)
            torch.cuda.synchronize()
            done = time.perf_counter() - t0
            lat.append(done - a)
            if i == warmup:
                first = a
        return dict(pct(lat), maps_s=(n - warmup) / (done - first))

    arena_gb = 64
    srv_cfgs = [dict(max_inflight=2, max_batch=1), dict(max_inflight=2, max_batch=8, group_ratio=2),
                dict(max_inflight=3, max_batch=4, group_ratio=2)]

    def serve(arr, cfg):
        srv = lf.Server(arena_gb << 30, dev, max_queue=n + 16, **cfg)
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = []
        for r, o, a in zip(reqs, outs, arr):
            wait_until(t0, a)
            tickets.append(srv.submit(r["views"], r["hyp"], r["params"], o))
        infos = [srv.wait(t) for t in tickets]
        st = srv.stats()
        srv.close()
        ok = all(i["status"] == 0 for i in infos)
        lat = [i["t_done"] - i["t_submit"] for i in infos]
        span = max(i["t_done"] for i in infos[warmup:]) - infos[warmup]["t_submit"]
        torch.cuda.synchronize()
        same = ok and all(torch.equal(a, b) for a, b in zip(outs, ref))
        sizes = [i["batch_size"] for i in infos[counted]]
        c = infos[counted]
        phase = {"queue_ms": float(np.mean([i["t_admit"] - i["t_submit"] for i in c]) * 1e3),
                 "plan_launch_ms": float(np.mean([i["t_launch"] - i["t_admit"] for i in c]) * 1e3),
                 "device_ms": float(np.mean([i["t_done"] - i["t_launch"] for i in c]) * 1e3)}
        return dict(pct(lat), maps_s=(n - warmup) / span, batches=st["batches"],
                    mean_batch=float(np.mean(sizes)), arena_peak_gb=st["arena_peak"] / 2**30,
                    identical_to_plain=bool(same), config=cfg, mean_phase=phase)

    rng = np.random.default_rng(12)
    gaps = rng.exponential(1.0, size=n)
    results = {}
    for rho in rates:
        rate = rho / mean_svc
        arr = np.cumsum(gaps / rate)
        pl = plain(arr)
        runs = [serve(arr, c) for c in srv_cfgs]
        results[rho] = dict(rate_per_s=rate, plain=pl, served_all=runs)
        log(f"[bench] rho {rho}: plain p50 {pl['p50_ms']:.2f} p99 {pl['p99_ms']:.2f} ms; served "
            + "; ".join(f"{r['config']}: p50 {r['p50_ms']:.2f} p99 {r['p99_ms']:.2f}"
                        for r in runs))
    del ws
    # the configuration with the lowest p99 at rho = 0.8, at every rate
    best = min(range(len(srv_cfgs)), key=lambda i: results[rates[0]]["served_all"][i]["p99_ms"])
    sweep = {str(rho): {"rate_per_s": v["rate_per_s"], "plain": v["plain"],
                        "served": v["served_all"][best]} for rho, v in results.items()}
    head = results[rates[0]]
    saturated = serve(np.zeros(n), srv_cfgs[best])
    return {"workload": "Poisson arrivals, requests uniform over the 5x5x96^2 u8 N=32, "
                        "9x9x512^2 N=100 and mixed 5x5x256^2 / 7x7x384^2 / 9x9x512^2 "
                        "(N 32..128) light fields",
            "requests": n, "warmup_requests": warmup, "rho": rates[0],
            "rate_per_s": head["rate_per_s"], "mean_alone_ms": mean_svc * 1e3,
            "served": head["served_all"][best], "plain": head["plain"],
            "served_all": head["served_all"], "sweep": sweep,
            "saturated_served_maps_s": saturated["maps_s"],
            "saturated_plain_maps_s": 1.0 / mean_svc,
            "server": dict(arena_gb=arena_gb, **srv_cfgs[best])}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="paper", choices=["paper", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the accuracy / boundary-less comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the request-loop measurement")
    ap.add_argument("--no-large", action="store_true", help="skip the large-workload measurement")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--serve-n", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--summarize-kernels", nargs=2, metavar=("STATS_CSV", "COMMAND"),
                    help="print a markdown summary of a rocprofv3 kernel-stats CSV and exit")
    ap.add_argument("--summarize-counters", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "WORKLOAD", "OUT_PREFIX"),
                    help="write OUT_PREFIX.json/.md from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of a --calib-copy run, and exit")
    ap.add_argument("--replay-plan", action="store_true",
                    help="only build the batched workload's plan and replay it 3 times")
    ap.add_argument("--summarize-plan-gaps", nargs=2, metavar=("TRACE_CSV", "COMMAND"),
                    help="print a markdown summary of a kernel trace of --replay-plan and exit")
    ap.add_argument("--summarize-stalls", nargs=2, metavar=("SQ_CSV", "TITLE"),
                    help="print the markdown wave-cycle breakdown of an SQ stall counter run "
                         "(see summarize_stalls) and exit")
    ap.add_argument("--summarize-units", nargs=4, metavar=("SQ_CSV", "TA_CSV", "TD_CSV", "TITLE"),
                    help="print a markdown table of per-kernel unit utilisation from three "
                         "rocprofv3 --pmc runs (see summarize_units) and exit")
    ap.add_argument("--commands", nargs="*", default=[],
                    help="the rocprofv3 commands recorded with --summarize-counters / -units")
    args = ap.parse_args()
    if args.summarize_kernels:
        print(summarize_kernel_stats(*args.summarize_kernels))
        return
    if args.summarize_plan_gaps:
        print(summarize_plan_gaps(*args.summarize_plan_gaps))
        return
    if args.summarize_stalls:
        sq, title = args.summarize_stalls
        print(f"# {title}\n\n" + summarize_stalls(sq, args.commands))
        return
    if args.summarize_units:
        sq, ta, td, title = args.summarize_units
        print(f"# {title}\n\n" + summarize_units(sq, ta, td, args.commands))
        return
    if args.summarize_counters:
        fetch, write, name, out = args.summarize_counters
        rec, md = summarize_counters(fetch, write, float(1 << 30), name, args.commands)
        json.dump(rec, open(out + ".json", "w"), indent=1)
        open(out + ".md", "w").write(f"# HBM traffic per launch (rocprofv3 counters): {name}\n\n"
                                     + md + "\n")
        print(md)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import lfsynth
    from paper_1907_13449_amd import lf

    dev = torch.device("cuda:0")
    if args.replay_plan:
        replay_plan(dev)
        return
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

    # the timed steps run without the stage-event hook; the same number of steps
    # is then run again with it, for the per-stage times
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    gpu_ms = float(ev[0].elapsed_time(ev[-1]))
    ms_per_step = gpu_ms / args.steps
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall * 1e3 / args.steps:.3f})")
    lf.profile_enable(True)
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    lf.profile_enable(False)
    stages = lf.profile_read()

    stage_ms = {k: v[0] / args.steps for k, v in stages.items()}
    stage_launches = {k: v[1] // args.steps for k, v in stages.items()}
    # the initial stage as a whole: its three timed parts, one kernel each
    parts = ("initial_cost", "initial_paths", "initial_sum_wta")
    stage_ms["sgm_initial"] = sum(stage_ms[k] for k in parts)
    stage_launches["sgm_initial"] = sum(stage_launches[k] for k in parts)

    px_bytes = 1 if lfd.views.dtype == np.uint8 else 4
    work = algorithmic_work(S, T, H, W, N, nv, px_bytes, cells_initial, cells_bounded,
                            p["sum_bits"])
    counters = load_counter_record(lfd.name)

    def counter_bytes(stage):
        ks = [k for k in STAGE_KERNELS.get(stage, []) if k in counters]
        if not ks:
            return None
        return sum(counters[k]["fetch_bytes"] + counters[k]["write_bytes"] for k in ks)

    stage_roofline = {}
    for name, wk in work.items():
        ms = stage_ms.get(name, 0.0)
        if ms <= 0:
            continue
        e = {"ms": ms, "launches": stage_launches.get(name, 0), "bytes": wk["bytes"],
             "achieved_gbs": wk["bytes"] / (ms * 1e-3) / 1e9,
             "frac_hbm": wk["bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "kernels": STAGE_KERNELS[name]}
        if "flop" in wk:
            e.update(flop=wk["flop"], achieved_tflops=wk["flop"] / (ms * 1e-3) / 1e12,
                     frac_fp32=wk["flop"] / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, bound="alu")
        else:
            e["bound"] = "hbm"
        tb = counter_bytes(name)
        e["traffic"] = tb
        e["traffic_ratio"] = tb / wk["bytes"] if tb and wk["bytes"] else None
        stage_roofline[name] = e

    # the dominant unit: the initial stage (Census cost volume, path costs, their sum
    # and WTA), its algorithmic bytes over the time of its three launches
    ini = stage_roofline["sgm_initial"]
    npaths = p["npaths"]
    kernel_model = {
        "note": "this design's own traffic per kernel (8-bit cost volume and path costs), "
                "not the algorithmic figure",
        "census_cost_volume_kernel": {"ms": stage_ms["initial_cost"],
                                      "bytes_per_cell": 1.0,
                                      "achieved_gbs": cells_initial / (stage_ms["initial_cost"]
                                                                       * 1e-3) / 1e9},
        "sgm_dense_paths_kernel": {"ms": stage_ms["initial_paths"],
                                   "bytes_per_cell": 1.0 + npaths,
                                   "achieved_gbs": (1.0 + npaths) * cells_initial /
                                   (stage_ms["initial_paths"] * 1e-3) / 1e9},
        "dense_sum_wta_rows_kernel": {"ms": stage_ms["initial_sum_wta"],
                                      "bytes_per_cell": float(npaths),
                                      "achieved_gbs": npaths * cells_initial /
                                      (stage_ms["initial_sum_wta"] * 1e-3) / 1e9},
    }
    for k, v in kernel_model.items():
        if isinstance(v, dict):
            v["frac"] = v["achieved_gbs"] / HBM_PEAK_GBS
            c = counters.get(k)
            v["traffic"] = c["fetch_bytes"] + c["write_bytes"] if c else None
    roofline = {"bound": "hbm", "achieved": ini["achieved_gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ini["frac_hbm"], "traffic": ini["traffic"],
                "traffic_ratio": ini["traffic_ratio"], "stage": "sgm_initial",
                "kernels": ["census_cost_volume_kernel", "sgm_dense_paths_kernel",
                            "dense_sum_wta_rows_kernel"],
                "launches": ini["launches"], "ms": ini["ms"],
                "bytes_per_cell": 12.0 + 18.0 / N, "cells": cells_initial,
                "bytes": ini["bytes"], "kernel_model": kernel_model}
    total_bytes = sum(wk["bytes"] for wk in work.values())
    all_k = [k for st in work for k in STAGE_KERNELS.get(st, [])]
    present = [k for k in all_k if k in counters]
    step_traffic = (sum(counters[k]["fetch_bytes"] + counters[k]["write_bytes"]
                        for k in present) if present else None)
    whole_step = {"bytes": total_bytes, "ms": ms_per_step,
                  "achieved_gbs": total_bytes / (ms_per_step * 1e-3) / 1e9,
                  "frac": total_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "traffic": step_traffic,
                  "traffic_ratio": step_traffic / total_bytes if step_traffic else None,
                  "note": "every stage's algorithmic bytes (the bounded cost's included, "
                          "although its bound is fp32 arithmetic) over the step time"}

    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    sum_t = "u16" if p["sum_bits"] == 16 else "u32"
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
        "dtype": f"f32+u8/u16/{sum_t}",
        "dtypes": {"views": "f32" if px_bytes == 4 else "u8",
                   "initial_cost_volume": "u8", "initial_path_costs": "u8 (u16 when "
                   "bits + P2 > 255)", "initial_sums": "u16 (in registers)",
                   "l2_cost": "f32", "bounded_cost": "u16", "bounded_path_costs": "u16",
                   "bounded_sums": sum_t, "disparity": "f32"},
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
        "whole_step": whole_step,
        "stage_roofline": stage_roofline,
        "paper_runtime": PAPER_RUNTIME,
    }
    if not args.no_quality:
        res["quality"] = quality_vs_boundless(lf, lfd, views, hyp, out, ms_per_step,
                                              cells_bounded, stream)
    del ws
    scenes = None
    if not (args.no_batch and args.no_serve) and args.workload == "paper":
        scenes = mixed_scenes(lfd, dev)
    if not args.no_batch and scenes is not None:
        res["batched"] = run_batched(scenes, args.batch_n, dev)
        res["batched_benchmark_shape"] = run_batched_benchmark_shape(views, hyp, p, 8, dev)
        torch.cuda.empty_cache()
    if not args.no_large and args.workload == "paper":
        res["large"] = run_large(dev)
        torch.cuda.empty_cache()
    if not args.no_serve and scenes is not None:
        res["served"] = run_served(scenes, args.serve_n, args.serve_warmup, dev)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle (3 whole light fields, one core)")
        small = lfsynth.workload("small") if args.workload == "paper" else None
        small_cells = None
        if small is not None:
            sv = torch.from_numpy(small.views).to(dev)
            sh = torch.from_numpy(small.hyp).to(dev)
            small_cells = request_cells(lf, dict(views=sv, hyp=sh, params=small.params))
        res["cpu_baseline"] = cpu_baseline(lfd, cells, small, small_cells)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
