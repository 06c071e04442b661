"""Builds libpa_amd.so (HIP kernels for gfx950 + the C-ABI host runtime) in-tree.

Usage: python -m paper_2511_20511_amd.build   (or build() from Python)

Every HIP source is compiled with -ffp-contract=off (the kernels spell out
each fused multiply-add they want, so every variant rounds identically) and
with packed FP32 instructions disabled.
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
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpa_amd.so")

# (source, object name, extra defines)
SOURCES = [(f, f, []) for f in ("api.cpp", "k_prep.hip", "k_fitness.hip", "k_ga.hip",
                                "k_kmeans.hip", "k_gen.hip", "solve.cpp", "server.cpp",
                                "k_exhaustive.hip", "k_peak.hip", "k_noalloc.hip",
                                "k_island.hip", "k_gen_wg.hip")]
# the unrolled generation kernels: one object per (cells, SE mode, form), so
# that they compile in parallel
SOURCES += [("k_gen_unrolled.hip", f"k_gen_L{L}_m{m}_{form}.hip",
             [f"-DPA_GEN_L={L}", f"-DPA_GEN_MODE={m}", f"-DPA_GEN_FORM={form}",
              f"-DPA_GEN_PERSIST={int(form == 'p')}"])
            for L in (37, 19, 7) for m in (0, 1) for form in ("x", "p")]
ARCH = "gfx950"


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def flags() -> list[str]:
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def _compile(unit) -> str:
    src, name, defines = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [_hipcc()] + flags() + defines + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
