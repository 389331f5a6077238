"""Build libkaze.so (HIP, gfx950) in the package directory.

Usage: ``python -m paper_1706_06750_amd.build``.  Cross-compiles on a machine
without a GPU; the shared library is written next to this file.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG_DIR)
LIB_PATH = os.path.join(PKG_DIR, "libkaze.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are kept out of the generated code on purpose.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(PKG_DIR, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass reports the device-only target feature as unknown
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    return res.returncode, err


def build(verbose: bool = False) -> str:
    """Compile every HIP source (one hipcc per source, in parallel) and link
    libkaze.so; returns the library path."""
    from concurrent.futures import ThreadPoolExecutor
    tag = ".tmp%d" % os.getpid()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG_DIR, "csrc")]
    objs = [os.path.join(PKG_DIR, "csrc", os.path.basename(f)[:-4] + tag + ".o") for f in sources()]
    jobs = [[HIPCC] + HIP_FLAGS + ["-c"] + inc + [f, "-o", o] for f, o in zip(sources(), objs)]
    workers = max(1, min(len(jobs), len(os.sched_getaffinity(0)), 16))
    tmp = LIB_PATH + tag
    try:
        with ThreadPoolExecutor(workers) as ex:
            results = list(ex.map(lambda c: _run(c, verbose), jobs))
        for (rc, err), cmd in zip(results, jobs):
            if rc != 0:
                raise RuntimeError("hipcc failed (%d) on %s:\n%s" % (rc, cmd[-3], err))
            if verbose and err.strip():
                print(err, file=sys.stderr)
        rc, err = _run([HIPCC] + HIP_FLAGS + ["-shared"] + objs + ["-o", tmp], verbose)
        if rc != 0:
            raise RuntimeError("link failed (%d):\n%s" % (rc, err))
        os.replace(tmp, LIB_PATH)
    finally:
        for f in objs + [tmp]:
            if os.path.exists(f):
                os.unlink(f)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
