"""Build step of the ZDA zone library: compiles the gfx950 HIP sources into
libzda.so next to this file (in-tree, so it travels with the repository)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", "zda_runtime.hip"), os.path.join(HERE, "csrc", "zda_kernels.hip")]
LIB = os.path.join(HERE, "libzda.so")
ARCH = os.environ.get("ZDA_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # contract a*b+c only inside one source expression, so that every kernel
    # built from the same update code rounds identically
    "-ffp-contract=on",
    # no packed FP32 instructions in the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libzda.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
