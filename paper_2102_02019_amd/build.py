"""Compiles the HIP sources of the package into liblabfm.so for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblabfm.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# gfx950 HIP flags: packed fp32 instructions are switched off for all device
# code. Floating-point contraction is left to the compiler except where a
# result must be rounded step by step (the stencil distance test and the
# error-free transformations), which switch it off locally.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
# weights.hip: LDS atomics are issued as they are written. The compiler's
# atomic optimizer would otherwise turn each pivot proposal (an LDS max from a
# few lanes) into a loop over the active lanes, a dozen instructions per lane,
# on the LU's critical path. The rows-in-registers kernel's column loops must
# unroll fully (its rows are register arrays indexed by the column); the
# default cost limit of a requested full unroll stops short at order 8.
FILE_FLAGS = {"weights.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
                               "-mllvm", "-pragma-unroll-threshold=1000000"]}
SOURCES = ["api.cpp", "tune_cache.cpp", "neighbours.hip", "weights.hip", "operators.hip", "tiles.hip", "adjoint.hip",
           "boundaries.hip", "lagrangian.hip", "morton.hip", "probe.hip"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *HIP_FLAGS, *FILE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


NODEGEN_SRC = os.path.join(HERE, "hostsrc", "place_nodes.c")
NODEGEN_LIB = os.path.join(HERE, "libnodegen.so")


def build_nodegen() -> str:
    """Host helper of the input generator (variable-resolution node sweep)."""
    tmp = NODEGEN_LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", NODEGEN_SRC, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {NODEGEN_SRC} failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, NODEGEN_LIB)
    return NODEGEN_LIB


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link liblabfm.so next to this file."""
    os.makedirs(OBJDIR, exist_ok=True)
    build_nodegen()
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
