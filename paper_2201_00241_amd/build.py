"""Build librh.so in place: host planner with g++, device code with hipcc (gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
CSRC = HERE / "csrc"
OUT = HERE / "librh.so"
BUILD = HERE.parent / "_build"
ROCM = Path(os.environ.get("ROCM_PATH", "/opt/rocm"))
HOST_SOURCES = ["network.cpp", "sparse_lu.cpp", "api.cpp", "tune.cpp"]
DEVICE_SOURCES = ["device.hip", "newton.hip", "dense.hip", "track.hip"]
# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _run(cmd):
    print(" ".join(str(c) for c in cmd), flush=True)
    subprocess.run([str(c) for c in cmd], check=True)


def build(verbose: bool = True) -> Path:
    BUILD.mkdir(exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        o = BUILD / (src + ".o")
        _run(["g++", *CXX_FLAGS, "-c", CSRC / src, "-o", o])
        objs.append(o)
    hipcc = ROCM / "bin" / "hipcc"
    for src in DEVICE_SOURCES:
        o = BUILD / (src + ".o")
        _run([hipcc, *HIP_FLAGS, "-c", CSRC / src, "-o", o])
        objs.append(o)
    tmp = OUT.with_suffix(".so.tmp")
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
