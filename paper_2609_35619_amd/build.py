"""Builds libcsplat.so (the HIP library behind include/csplat.h) for gfx950.

Each .hip translation unit is compiled with hipcc in parallel and linked into
one shared library next to this file.  Packed-FP32 instruction selection is
disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcsplat.so")
ARCH = os.environ.get("CSPLAT_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["abi.hip", "scene.hip", "pair_fp32.hip", "precision.hip", "serve.hip", "segment.hip", "rrt.hip", "ply.cpp",
           "sched.cpp"]

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
         "-I", os.path.join(ROOT, "include")]

# Per-source extra flags.  The MFMA label kernel reads every accumulator
# element right after its product; with the accumulators in ordinary VGPRs
# (the backend otherwise picks the AccVGPR file) no v_accvgpr_read copies
# are needed, and the kernel needs fewer registers.
SOURCE_FLAGS = {"precision.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src: str, build_dir: str = BUILD, defines=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *SOURCE_FLAGS.get(src, []), *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source and link `out`.  `defines` (NAME=VALUE strings)
    override the launch-shape constants, for tuning sweeps."""
    build_dir = BUILD if out == LIB else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, defines), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


SCHED_TEST_LIB = os.path.join(HERE, "libcsplat_sched.so")


def build_sched_test_lib(verbose: bool = False) -> str:
    """The serving scheduler alone, host compiler only, for CPU tests."""
    tmp = SCHED_TEST_LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", "-Wextra",
           os.path.join(CSRC, "sched.cpp"), os.path.join(CSRC, "sched_capi.cpp"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed on the scheduler:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SCHED_TEST_LIB)
    if verbose:
        print("built", SCHED_TEST_LIB)
    return SCHED_TEST_LIB


if __name__ == "__main__":
    build_sched_test_lib(verbose=True)
    build(verbose=True)
    sys.exit(0)
