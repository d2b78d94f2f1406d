"""Build libmsft.so in-tree: host geometry and ABI with g++, kernels with hipcc for gfx950."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmsft.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

# Packed FP32 VALU forms are kept out of every device build.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter"]

SOURCES_HOST = ["geometry.cpp", "abi.cpp"]
SOURCES_HIP = ["kernels.hip", "gauss.hip", "backward.hip", "render.hip", "detector.hip",
               "noalloc.hip", "sepg.hip", "peaks.hip"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    inc = ["-I" + INCLUDE, "-I" + CSRC]
    for src in SOURCES_HOST:
        obj = os.path.join(BUILD, src + ".o")
        # -ffp-contract=off: the q map must be reproducible bit for bit
        extra = ["-ffp-contract=off"]
        if src == "abi.cpp":
            extra += ["-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")]
        _run(["g++", *HOST_FLAGS, *extra, *inc, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in SOURCES_HIP:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
          "-Wl,-rpath," + os.path.join(ROCM, "lib")], verbose)
    os.replace(tmp, LIB)
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
