"""Build libtc.so (HIP, gfx950) in-tree with hipcc.

Runs without a GPU: hipcc cross-compiles the device code for gfx950.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "csrc")
LIB = os.path.join(_HERE, "libtc.so")
SOURCES = ["tc_kernels.hip", "tc_api.hip", "tc_parse.hip", "tc_probe.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-result",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, *extra,
           *[os.path.join(_CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
