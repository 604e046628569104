"""Build the HIP library (libmhd.so) for gfx950 in-tree with hipcc.

Usage: python -m paper_0908_4362_amd.build  (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmhd.so")
# (source, extra flags): the FP64 kernels are built without FMA contraction so
# that they round exactly as the CPU oracle does; the FP32 kernels contract a
# multiply and an add only within one source expression, so every expression
# rounds the same wherever the unrolled marching loops place it and the chunk
# layout of a launch never changes a result
SOURCES = [("mhd_kernels_f64.hip", ["-ffp-contract=off"]), ("mhd_kernels_f32.hip", ["-ffp-contract=on"]), ("mhd_api.hip", []),
           ("mhd_batch.hip", []), ("mhd_server.hip", [])]
ARCH = "gfx950"

# Packed FP32 instructions are kept out of the device code: the compiler may
# only emit scalar or vector FP32 arithmetic.
HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False, extra_flags=None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    for src, flags in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc, *HIPFLAGS, *flags, *(extra_flags or []), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
