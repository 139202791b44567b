"""Build libdtwmi.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2307_04904_amd.csrc.build   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(OUT_DIR, "libdtwmi.so")
SOURCES = ["dtw_stage.hip", "dtw_lane.hip", "dtw_lane_rb.hip", "dtw_lane_split.hip", "dtw_strip.hip", "dtw_strip_f64.hip", "dtw_cyclic.hip", "dtw_cluster.hip", "dtw_path.hip", "dtw_api.hip"]
ARCH = os.environ.get("DTWMI_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # exact IEEE ops as written: no contraction (the Kahan and FP64 kernels rely on it)
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


NOISE = ("packed-fp32-ops' is not a recognized feature", "argument unused during compilation")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (res.stdout + res.stderr).splitlines() if l.strip() and not any(n in l for n in NOISE)]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed (%d): %s\n%s" % (res.returncode, " ".join(cmd), "\n".join(msgs)))
    if verbose and msgs:
        print("\n".join(msgs))


# per-source flags: the FP64 strips produce no NaN, so they drop signalling-NaN handling
EXTRA = {"dtw_strip_f64.hip": ["-fno-honor-nans", "-mno-amdgpu-ieee"]}


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source to an object (in parallel), then link the shared library."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OUT_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", HERE]
    tag = "%d" % os.getpid()
    objs = [os.path.join(OUT_DIR, os.path.splitext(s)[0] + ".o." + tag) for s in SOURCES]
    cmds = [["hipcc"] + FLAGS + EXTRA.get(s, []) + inc + ["-c", os.path.join(HERE, s), "-o", o]
            for s, o in zip(SOURCES, objs)]
    jobs = jobs or min(len(cmds), os.cpu_count() or 1, 8)
    try:
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            for f in [pool.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp" + tag
        _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
