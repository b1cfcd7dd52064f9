"""Build the gfx950 shared library libec_hip.so in-tree with hipcc.

Flags: FP64 without contraction (-ffp-contract=off; every fused multiply-add
is an explicit fma()), packed-FP32 instructions disabled for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libec_hip.so")
SOURCES = [os.path.join(CSRC, "ec_kernels.hip"), os.path.join(CSRC, "ec_observe.hip"),
           os.path.join(CSRC, "ec_static.hip"), os.path.join(CSRC, "ec_api.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False) -> str:
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-command-line-argument",
           "-I", os.path.join(HERE, "..", "include"),
           "-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
