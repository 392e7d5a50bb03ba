"""Build the HIP library libfhe_mi355x.so in place (gfx950 only)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfhe_mi355x.so")
SOURCES = ["api.hip", "kernels.hip", "ops.hip", "encode.cpp", "boot.cpp"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    """Compile every source into the shared library; returns its path."""
    cmd = [
        hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions are kept out of every code object
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # the reconstruction and lift kernels unroll their k-block and tile loops fully
        "-mllvm", "-pragma-unroll-threshold=1000000",
        "-Wno-unused-result", "-Wno-unused-value", "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
        "-o", LIB + ".tmp",
    ] + [os.path.join(HERE, "csrc", s) for s in SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
