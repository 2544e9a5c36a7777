"""Builds libmlswe.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmlswe.so")
CSRC = os.path.join(HERE, "csrc")
# (source, extra flags): the fast sweeps may contract a*b+c into fma
SRCS = [(os.path.join(CSRC, "mlswe_kernels.hip"), []),
        (os.path.join(CSRC, "mlswe_sweeps_fast.hip"), ["-ffp-contract=fast"]),
        (os.path.join(CSRC, "mlswe_adjoint.hip"), []),
        (os.path.join(CSRC, "mlswe_layers.hip"), []),
        (os.path.join(CSRC, "mlswe_lib.cpp"), []),
        (os.path.join(CSRC, "mlswe_launch.cpp"), []),
        (os.path.join(CSRC, "mlswe_regrid.cpp"), []),
        (os.path.join(CSRC, "mlswe_advance.cpp"), []),
        (os.path.join(CSRC, "mlswe_adjoint_host.cpp"), []),
        (os.path.join(CSRC, "mlswe_tuning.cpp"), [])]
HDRS = [os.path.join(HERE, "csrc", "mlswe_kernels.hpp"), os.path.join(HERE, "csrc", "mlswe_device.hpp"),
        os.path.join(HERE, "csrc", "mlswe_host.hpp"),
        os.path.join(HERE, "csrc", "mlswe_layers.hpp"),
        os.path.join(ROOT, "include", "mlswe.h")]
ARCH = os.environ.get("MLSWE_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]
# exact builds: FP64 results must not depend on contraction choices
EXACT = ["-ffp-contract=off"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src, extra in SRCS:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc] + FLAGS + (extra if extra else EXACT) + ["-c", "-x", "hip", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def build_test_lib(src: str, out: str, verbose: bool = False) -> str:
    """A test-only shared library from one HIP source that includes the
    library's device headers (exact-build flags)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc] + FLAGS + EXACT + ["-I" + CSRC, "-shared", "-x", "hip", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
