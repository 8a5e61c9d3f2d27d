"""Build step of the ZDA zone library: compiles the gfx950 HIP sources into
libzda.so next to this file (in-tree, so it travels with the repository)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", "zda_runtime.hip"), os.path.join(HERE, "csrc", "zda_kernels.hip")]
LIB = os.path.join(HERE, "libzda.so")
# the design surrogate's kernels (BF16 MFMA GEMM and training pieces)
SUR_SOURCES = [os.path.join(HERE, "csrc", "zsur_kernels.hip")]
SUR_LIB = os.path.join(HERE, "libzsur.so")
ARCH = os.environ.get("ZDA_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    # contract a*b+c only inside one source expression, so that every kernel
    # built from the same update code rounds identically
    "-ffp-contract=on",
    # no packed FP32 instructions in the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _build_one(sources, lib, verbose):
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *FLAGS, "-o", tmp, *sources]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building %s" % os.path.basename(lib))
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Builds libzda.so (zone library) and libzsur.so (surrogate kernels)."""
    _build_one(SUR_SOURCES, SUR_LIB, verbose)
    return _build_one(SOURCES, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
