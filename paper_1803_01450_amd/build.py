"""Builds libmlswe.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmlswe.so")
SRCS = [os.path.join(HERE, "csrc", "mlswe_kernels.hip"), os.path.join(HERE, "csrc", "mlswe_adjoint.hip"),
        os.path.join(HERE, "csrc", "mlswe_lib.cpp")]
HDRS = [os.path.join(HERE, "csrc", "mlswe_kernels.hpp"), os.path.join(HERE, "csrc", "mlswe_device.hpp"),
        os.path.join(ROOT, "include", "mlswe.h")]
ARCH = os.environ.get("MLSWE_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # FP64 results must not depend on contraction choices
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + FLAGS
    for src in SRCS:
        cmd += ["-x", "hip", src]
    cmd += ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
