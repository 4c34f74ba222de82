"""Builds libfftu.so (HIP kernels for gfx950 plus the C-ABI host code) in-tree.

Run ``python -m paper_2203_11795_amd.build`` or call :func:`build`. The result
sits next to this file, where :mod:`paper_2203_11795_amd.fftu` loads it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfftu.so")
ARCH = "gfx950"

SOURCES = ["fftu_api.cpp", "fftu_kernels.hip", "fftu_line.hip", "fftu_exchange.hip", "fftu_group.hip", "fftu_pair.hip", "fftu_long.hip",
           "fftu_lastx_f32.hip", "fftu_lastx_f64.hip", "fftu_batch.hip", "fftu_fill.hip", "fftu_pointwise.hip", "fftu_mixed.hip", "fftu_scratch.hip", "fftu_gcyclic.hip", "fftu_real.hip",
           "fftu_r2r.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)


def build(verbose: bool = False, resource_usage: bool = False, jobs: int = 0) -> str:
    """Compile every source for gfx950 (in parallel, `jobs` at a time; 0 = one per
    source, at most 8) and link libfftu.so; returns its path."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if resource_usage and src.endswith(".hip"):
            cmd.append("-Rpass-analysis=kernel-resource-usage")
        cmds.append(cmd)
        objs.append(obj)
    workers = jobs if jobs > 0 else min(8, len(cmds))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        for fut in [pool.submit(_run, c, verbose or resource_usage) for c in cmds]:
            fut.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, resource_usage="--usage" in sys.argv))
