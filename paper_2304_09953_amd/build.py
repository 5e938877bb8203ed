"""Build steps for the native parts of the package.

* ``build_library()``: the HIP kernels and the C ABI (``include/ligate_dock.h``)
  into ``libligate.so``, for gfx950 only.
* ``build_inputs()``: the seeded input generator (plain C) into
  ``inputs/libligate_inputs.so``.
"""
from __future__ import annotations

import glob
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB_PATH = os.path.join(PKG, "libligate.so")
INPUTS_LIB = os.path.join(PKG, "inputs", "libligate_inputs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instruction selection is switched off for every HIP source: some packed FP32 forms
# have given silently wrong results.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-L", "/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def build_library(verbose: bool = False, extra=()) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, *HIP_FLAGS, *extra, "-o", tmp, *srcs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stdout + r.stderr)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_inputs(verbose: bool = False) -> str:
    src = os.path.join(PKG, "inputs", "gen.c")
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-shared", "-fPIC", "-o", INPUTS_LIB, src, "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    return INPUTS_LIB
