"""Compile the HIP library (gfx950) in-tree: paper_1701_03549_amd/libfiregpu.so."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfiregpu.so")
SOURCES = [os.path.join(CSRC, "fire_kernels.hip"), os.path.join(CSRC, "fire_abi.cpp"),
           os.path.join(CSRC, "surrogate.hip"), os.path.join(CSRC, "probe.hip")]
ARCH = os.environ.get("FIREGPU_ARCH", "gfx950")


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def compile_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            # loadable by the HIP runtime bundled with PyTorch as well
            "-mcode-object-version=5",
            "-ffp-contract=off", "-fno-fast-math",
            # keep the compiler from forming packed fp32 arithmetic
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Always recompiles (this is the build check); returns the library path."""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        cmd = [hipcc(), "-c", "-x", "hip"] + compile_flags() + ["-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-mcode-object-version=5", "-shared", "-fPIC",
           "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
