"""Build libmpmc.so in-tree with hipcc for gfx950.

    python -m paper_1211_1646_amd.build

Flags: -O3, no floating-point contraction (bit-exact with the CPU oracle's
specification), packed-FP32 instructions disabled, position-independent
shared library exporting the C ABI of include/mpmc.h and
include/mpmc_sphere.h.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmpmc.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("mpmc_kernels.hip", "mpmc_mlp.hip",
                                                       "mpmc_api.cpp", "sphere_kernels.hip",
                                                       "sphere_api.cpp")]
ARCH = os.environ.get("MPMC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags():
    return ["-O3", "-std=c++17", "--offload-arch=%s" % ARCH, "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    """Compile every source and link libmpmc.so (always recompiles)."""
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"]
        cmd = [hipcc()] + flags() + lang + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=%s" % ARCH, "-shared", "-fPIC",
           "-Wl,--version-script=%s" % os.path.join(HERE, "csrc", "libmpmc.map"), "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
