"""Build libwb.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Every source is compiled to an object under ``_build/`` in parallel and
linked into ``paper_2603_05493_amd/libwb.so``.  Packed FP32 instructions are
disabled for the device code (``-packed-fp32-ops``).  A separate
``libwb_peak.so`` holds the benchmark's FP32 FMA-rate probe.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libwb.so")
PEAK_LIB = os.path.join(PKG, "libwb_peak.so")
PEAK_SOURCES = ["valu_peak.hip"]

SOURCES = ["wb_host.cpp", "fk.hip", "rnea.hip", "selfcoll.hip", "misc.hip", "fused.hip", "bspline.hip",
           "kinematics.hip", "edt.hip", "edt_scratch.hip", "tree_kernels.hip"]
ARCH = os.environ.get("WB_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found; set ROCM_PATH")


def flags():
    return ["-x", "hip", "-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *flags(), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + PEAK_SOURCES
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    _link([objs[s] for s in SOURCES], LIB)
    _link([objs[s] for s in PEAK_SOURCES], PEAK_LIB)
    if verbose:
        print(f"built {LIB} and {PEAK_LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
