"""Builds liblf.so (the HIP kernels and the C ABI of include/lf.h) for gfx950.

    python -m paper_1907_13449_amd.build [--incremental]

Compiles every csrc/*.hip to an object (in parallel, one hipcc per file) under
_build/ and links them into paper_1907_13449_amd/liblf.so.  Floating-point
contraction is off (-ffp-contract=off): the l2 cost, the Sobel threshold and the
sub-pixel step are float32 expressions whose every rounding is written out (fmaf
where a fused multiply-add is meant), so that the quantised integer costs are
decided exactly as specified.  Packed-FP32 instructions are disabled for the
device code.  --incremental recompiles only sources newer than their object (or
than a header); the default rebuilds everything.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblf.so")
OBJ_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("LF_OFFLOAD_ARCH", "gfx950")
# hipcc's host pass does not know the packed-fp32 feature and says so; harmless
_NOISE = "is not a recognized feature for this target"


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def headers():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.h")) +
                  glob.glob(os.path.join(ROOT, "include", "*.h")))


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def compile_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


def command(out=LIB):
    """One hipcc call that compiles and links every source (for reference)."""
    return [_hipcc(), *compile_flags(), "-shared", "-o", out, *sources()]


def _obj(src):
    return os.path.join(OBJ_DIR, os.path.basename(src)[:-4] + ".o")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if _NOISE not in l)
    return res.returncode, err


def build(verbose: bool = False, force: bool = True, jobs: int = 8) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    newest_header = max(os.path.getmtime(h) for h in headers())
    todo = []
    for src in sources():
        obj = _obj(src)
        stale = (force or not os.path.exists(obj) or
                 os.path.getmtime(obj) < max(os.path.getmtime(src), newest_header))
        if stale:
            todo.append(src)

    def one(src):
        cmd = [_hipcc(), *compile_flags(), "-c", "-o", _obj(src), src]
        if verbose:
            print(" ".join(cmd), flush=True)
        return src, *_run(cmd)

    errors = []
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        for src, rc, err in ex.map(one, todo):
            if rc != 0:
                errors.append(f"{os.path.basename(src)}:\n{err}")
            elif verbose and err.strip():
                print(err, file=sys.stderr)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    link = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
            *[_obj(s) for s in sources()]]
    if verbose:
        print(" ".join(link), flush=True)
    rc, err = _run(link)
    if rc != 0:
        raise RuntimeError(f"link failed ({rc}):\n{err}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, force="--incremental" not in sys.argv[1:]))
