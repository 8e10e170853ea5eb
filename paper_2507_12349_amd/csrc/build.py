"""Build libcos.so for gfx950 with hipcc (cross-compiles without a GPU).

    python paper_2507_12349_amd/csrc/build.py

Writes paper_2507_12349_amd/libcos.so (in-tree, next to the Python binding).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
OUT = os.path.join(PKG, "libcos.so")
SOURCES = ["cos_level.hip", "cos_sub.hip", "cos_kernels.hip", "cos_mc.hip", "cos_cdet.hip", "cos_static.hip", "cos_count.hip", "libcos.cpp"]
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unknown-pragmas",
]


def build(verbose: bool = False, extra=()) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, *extra, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
