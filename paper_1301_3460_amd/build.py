"""Build ``liblgf.so`` (HIP, gfx950) in-tree with hipcc.

The library is a plain shared object with a C ABI (``include/lgf.h``); the
Python binding loads it with ctypes.  Run ``python -m paper_1301_3460_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblgf.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("sweep.hip", "su2.hip", "fft_f64.hip", "fft_f32.hip", "api.cpp")]
ARCH = os.environ.get("LGF_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    # contract multiply-adds only within one expression, so identical source
    # expressions round identically wherever they are inlined
    "-ffp-contract=on",
]


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel, one hipcc per translation unit) and
    link liblgf.so.  Always recompiles."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in SOURCES]

    def compile_one(pair):
        src, obj = pair
        cmd = ["hipcc", *HIPCC_FLAGS, "-c", "-x", "hip", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        list(ex.map(compile_one, zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
