"""Build the HIP library libexactmap.so for gfx950 (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libexactmap.so")

SOURCES = ["em_primitives.hip", "em_geometry.hip", "em_pairs.hip", "em_integrate.hip", "em_reduce.hip",
           "em_pseudo.hip", "em_table.hip", "em_voronoi.hip", "em_noalloc.hip", "em_api.cpp", "em_serve.cpp",
           "em_tune.cpp"]

# Packed FP32 instructions are disabled for all device code.
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", "-x", "hip"] + FLAGS + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


CALIB_SRC = os.path.join(CSRC, "calib", "em_calib.hip")
CALIB_LIB = os.path.join(OUT_DIR, "libemcalib.so")


def build_calib() -> str:
    """The benchmark's VALU calibration kernel (a separate library; not part of the mapping ABI)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = CALIB_LIB + ".tmp"
    cmd = ["hipcc", "-x", "hip"] + FLAGS + ["-shared", CALIB_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"calibration build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, CALIB_LIB)
    return CALIB_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    build_calib()
    if verbose:
        print("built", LIB, "and", CALIB_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
