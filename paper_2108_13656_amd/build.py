"""Builds the HIP library ``libdecolor.so`` in-tree for gfx950.

Run as ``python -m paper_2108_13656_amd.build``; the package loads the result
and never compiles anything itself.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdecolor.so")
SOURCES = [os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "runtime.cpp")]
ARCH = "gfx950"

# Packed FP32 (v_pk_*_f32) is switched off for every HIP translation unit.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "--offload-arch=" + ARCH]


# roctx: named host ranges around the entry points for rocprofv3's marker trace.
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# Memory-ceiling kernels of the benchmark (no part of libdecolor.so).
CEIL_LIB = os.path.join(HERE, "libdc_ceilings.so")
CEIL_SOURCES = [os.path.join(CSRC, "ceilings.hip")]


def build(verbose=False):
    """Compiles every source into libdecolor.so, and the benchmark's
    memory-ceiling kernels into libdc_ceilings.so (always recompiles)."""
    _compile(SOURCES, LIB, LIBS, verbose)
    _compile(CEIL_SOURCES, CEIL_LIB, [], verbose)
    return LIB


def _compile(sources, lib, libs, verbose):
    out_tmp = lib + ".tmp"
    cmd = [hipcc()] + HIP_FLAGS + ["-shared", "-o", out_tmp] + sources + libs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass reports the device-only feature flag as unknown; drop that noise.
    noise = "is not a recognized feature for this target"
    log = "\n".join(l for l in res.stdout.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + log)
    if verbose and log.strip():
        print(log)
    os.replace(out_tmp, lib)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
