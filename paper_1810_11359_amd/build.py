"""Build libism.so (HIP kernels for gfx950 + C ABI host code) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libism.so")
SOURCES = [os.path.join(CSRC, "ism_device.hip"), os.path.join(CSRC, "ism_diffuse.hip"),
           os.path.join(CSRC, "ism_filter.hip"), os.path.join(CSRC, "ism_filter_fft.hip"),
           os.path.join(CSRC, "ism_noalloc.hip"),
           os.path.join(CSRC, "ism_host.cpp")]
HEADERS = [os.path.join(CSRC, "ism_internal.h"), os.path.join(CSRC, "ism_math.h"), os.path.join(ROOT, "include", "ism.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # FMA contraction only where written explicitly (error-free transforms rely on it)
    "-ffp-contract=off",
    # no packed-FP32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile every source into paper_1810_11359_amd/libism.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def asm(out_path: str) -> str:
    """Device assembly of the kernels (for inspection)."""
    cmd = [HIPCC, *[f for f in FLAGS if f not in ("-shared", "-fPIC")], "--cuda-device-only", "-S",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, SOURCES[0], "-o", out_path]
    subprocess.check_call(cmd)
    return out_path


if __name__ == "__main__":
    # python -m paper_1810_11359_amd.build [--asm OUT.s]
    build(verbose=True)
    if len(sys.argv) > 2 and sys.argv[1] == "--asm":
        print(asm(sys.argv[2]))
