"""Build libpa.so (HIP for gfx950) in-tree.

Usage: python -m paper_1805_02372_amd.build   (or build() from Python)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpa.so")
ARCH = os.environ.get("PA_OFFLOAD_ARCH", "gfx950")

SOURCES = ["conv_fp32.hip", "conv_fp64.hip", "conv_fp32_p3.hip", "conv_fp32_p5.hip", "conv_fp32_p7.hip",
           "conv_fp64_p3.hip", "conv_fp64_p5.hip", "conv_fp64_p7.hip", "ntt.hip", "direct.hip", "classes.cpp",
           "engine.cpp", "noalloc.cpp", "stream.cpp", "serving.cpp", "tuner.cpp", "planner.cpp", "tables.cpp"]

# Packed FP32 instructions are disabled for all device code.  Code object v5
# loads in every ROCm 6/7 runtime, including the one PyTorch bundles.  Atomics
# on one address from a whole wave are combined with DPP reductions (the
# default combines them lane by lane in a scalar loop).
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-atomic-optimizer-strategy=DPP",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return h


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, *os.environ.get("PA_EXTRA_HIPCC_FLAGS", "").split()]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every HIP/C++ source and link libpa.so.  Always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-mcode-object-version=5", "-o", tmp, *objs,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
