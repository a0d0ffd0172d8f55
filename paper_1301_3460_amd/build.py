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


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer build (the CPU
# part of every translation unit only; device code is compiled as usual):
# liblgf_san.so, for host-only checks of the C ABI, loaded in a process that
# preloads clang's shared ASan runtime (see sanitizer_runtime()).
SAN_FLAGS = ["-Xarch_host", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]
SAN_LINK = ["-shared-libsan", "-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-fsanitize=undefined"]
LIB_SAN = os.path.join(HERE, "liblgf_san.so")


def sanitizer_runtime() -> str:
    """Path of clang's shared ASan runtime that a process loading
    liblgf_san.so must preload."""
    out = subprocess.run(["hipcc", "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True, check=True).stdout.strip()
    if not os.path.isabs(out):
        rd = subprocess.run(["hipcc", "-print-resource-dir"], capture_output=True, text=True,
                            check=True).stdout.strip()
        out = os.path.join(rd, "lib", "linux", "libclang_rt.asan-x86_64.so")
    return out


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source (in parallel, one hipcc per translation unit) and
    link liblgf.so (sanitize: liblgf_san.so with host-side ASan/UBSan).
    Always recompiles."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    lib = LIB_SAN if sanitize else LIB
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in SOURCES]
    extra = SAN_FLAGS if sanitize else []

    def compile_one(pair):
        src, obj = pair
        cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-c", "-x", "hip", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        list(ex.map(compile_one, zip(SOURCES, objs)))
    tmp = lib + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *(SAN_LINK if sanitize else []),
           *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
