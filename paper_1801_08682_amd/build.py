"""Build libadg.so (the ADER-DG kernels and the C ABI) and libadg_peaks.so
(roofline measurement kernels) for gfx950 in-tree with hipcc (parallel, one
object per unit).

Usage: python -m paper_1801_08682_amd.build [-j JOBS]
"""

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libadg.so")
PEAKS_LIB = os.path.join(HERE, "libadg_peaks.so")

UNITS = ["api.hip", "tables.cpp", "inst_advection.hip", "inst_euler.hip",
         "inst_acoustic.hip", "inst_elastic.hip"]
PEAKS_UNITS = ["peaks.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are switched off for every device compile.  The
# matrix-core instructions write their results to ordinary VGPRs (gfx950's
# unified register file) rather than AGPRs, which saves the copies back and
# keeps the bfloat16 predictor at three waves per SIMD.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-mllvm", "-amdgpu-mfma-vgpr-form",
                "-I", os.path.join(ROOT, "include")]


def _compile(unit):
    src = os.path.join(CSRC, unit)
    obj = os.path.join(BUILD, unit + ".o")
    cmd = [HIPCC] + DEVICE_FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, lib)


def build(jobs=None, verbose=False):
    """Compile every unit and link both libraries; returns libadg.so's path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, UNITS + PEAKS_UNITS))
    _link(objs[:len(UNITS)], LIB)
    _link(objs[len(UNITS):], PEAKS_LIB)
    if verbose:
        print("built", LIB, PEAKS_LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    build(a.j, verbose=True)
    sys.exit(0)
