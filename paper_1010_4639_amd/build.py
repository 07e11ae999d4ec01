"""Build the HIP library libcgmi.so in-tree for gfx950.

plan.cpp is plain host C++ (g++); kernels.hip, batch.hip, fem.hip and capi.cpp go through hipcc
with packed-FP32 instructions disabled (-packed-fp32-ops), then everything is
linked into one shared library next to this file.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcgmi.so")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    subprocess.run(cmd, check=True)


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    o = os.path.join(BUILD, "plan.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", os.path.join(CSRC, "plan.cpp"), "-o", o])
    objs.append(o)
    for src in ("kernels.hip", "batch.hip", "fem.hip", "capi.cpp"):
        o = os.path.join(BUILD, src.split(".")[0] + ".o")
        _run([HIPCC, *HIP_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
