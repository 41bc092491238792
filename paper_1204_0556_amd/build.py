"""Build the HIP library liblpdec.so for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblpdec.so")
SOURCES = ["lpdec_kernels.hip", "lpdec_aux.hip", "lpdec_host.cpp", "lpdec_aux_host.cpp", "lpdec_server.cpp",
           "lpdec_noalloc.hip"]
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no implicit FMA contraction: every fused multiply-add is an explicit fmaf,
    # so all kernel forms round identically
    "-ffp-contract=off",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        # The decoder kernels only ever compute on finite values (frames with a
        # non-finite LLR are detected from the bit pattern and never decoded), so
        # min/max need no NaN-quieting of their inputs.
        extra = ["-fno-honor-nans"] if src == "lpdec_kernels.hip" else []
        cmd = ["hipcc", *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
