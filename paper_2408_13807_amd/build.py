"""Build libire.so (HIP for gfx950) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIB_DIR, "libire.so")

SOURCES = ["ire_trace.hip", "ire_api.cpp", "ire_batch.cpp", "sur_kernels.hip", "sur_api.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


# the vector-ALU issue-rate tool behind the tracer's roofline peak (profiling only)
VALU_RATE = os.path.join(LIB_DIR, "valu_rate")


def build(verbose: bool = False) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip",
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    tool = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops", os.path.join(CSRC, "valu_rate.hip"), "-o", VALU_RATE + ".tmp"]
    if verbose:
        print(" ".join(tool), flush=True)
    subprocess.check_call(tool)
    os.replace(VALU_RATE + ".tmp", VALU_RATE)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
