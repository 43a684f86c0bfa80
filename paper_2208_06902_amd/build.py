"""Build libipls.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "ipls_lib.hip")
# host-only parts of the library: the batched form's autotuner and the request server
HOST_SRCS = [os.path.join(HERE, "csrc", "ipls_tune.cpp"), os.path.join(HERE, "csrc", "ipls_server.cpp")]
LIB = os.path.join(HERE, "libipls.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every fp64 operation is rounded where it is written: no FMA contraction, no fast math
    "-ffp-contract=off", "-fno-fast-math",
    # no packed fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, SRC, *HOST_SRCS, "-lpthread", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
