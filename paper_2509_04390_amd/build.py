"""Build librta.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "rta.hip")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librta.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # packed-FP32 VALU ops stay off: the compiler still vectorizes, but never
    # emits the packed add/mul/fma forms
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build_library(extra_flags=(), out: str = LIB) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, *extra_flags, "-I", INCLUDE,
           "-I", os.path.join(PKG, "csrc"), SRC, "-o", out + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_library())
