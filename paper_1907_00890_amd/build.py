"""Build libvofpoisson.so (HIP, gfx950) in-tree.

    python paper_1907_00890_amd/build.py     # or __graft_entry__.build()

Compiles every source under csrc/ with hipcc for gfx950 and links one shared
library next to this file.  Packed FP32 instructions are disabled for all
device code (-packed-fp32-ops); hipcc's host pass warns that it does not know
that feature, which is harmless.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libvofpoisson.so")

# (source, parts): a source with several parts is compiled once per part with
# -DVP_PART=k (each object holds a share of its entry points, so the template
# instantiations of one file spread over parallel jobs).  Heaviest first
# (compiled in parallel, in this order).
SOURCES = [("transforms_x.hip", 3), ("transforms_y.hip", 2), ("transforms_z.hip", 2),
           ("zsolve.hip", 2), ("stencils.hip", 1), ("advect.hip", 1), ("plan.cpp", 1),
           ("serve.cpp", 1),
           ("plan_check.cpp", 1)]
JOBS = [(src, k if n > 1 else 0) for src, n in SOURCES for k in range(1, n + 1)]
ARCH = os.environ.get("VP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libvofpoisson)")


def common_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-pthread",
        "-I", INCLUDE, "-I", CSRC,
    ]


def _compile(job) -> str:
    src, part = job
    stem = os.path.splitext(src)[0] + (f".p{part}" if part else "")
    obj = os.path.join(BUILD, stem + ".o")
    cmd = [hipcc()] + common_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    if part:
        cmd.append(f"-DVP_PART={part}")
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {stem}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile all sources and link libvofpoisson.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    workers = min(len(JOBS), max(1, os.cpu_count() or 2))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, JOBS))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
