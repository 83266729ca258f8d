"""Builds the gfx950 HIP library ``librtc.so`` in-tree with hipcc.

Each source is compiled to an object in its own hipcc process (in parallel),
then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librtc.so")
SOURCES = ["rtc_api.hip", "rtc_kernels.hip", "horizontal_kernels.hip", "pipe_api.hip", "pipe_kernels.hip",
           "mlp_api.hip", "mlp_kernels.hip"]

# -packed-fp32-ops: keep hipcc from fusing float pairs into packed FP32 VALU ops.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm install required to build librtc.so)")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compiles every HIP source into ``librtc.so`` next to this file; returns its path."""
    cc = hipcc()
    jobs = jobs or min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with tempfile.TemporaryDirectory(prefix="rtc_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[cc, *HIPCC_FLAGS, "-c", "-o", o, os.path.join(CSRC, s)] for s, o in zip(SOURCES, objs)]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(jobs) as pool:
            results = list(pool.map(run, cmds))
        for cmd, r in zip(cmds, results):
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed ({' '.join(cmd)}):\n{r.stderr}")
            if verbose and r.stderr.strip():
                lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
                if lines:
                    print("\n".join(lines), flush=True)
        tmp = LIB + ".tmp"
        link = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
