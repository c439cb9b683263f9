"""Build libslp.so for gfx950 in-tree (paper_1305_3162_amd/_lib/libslp.so).

Usage: python -m paper_1305_3162_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libslp.so")

SOURCES = ["slp_kernels.hip", "slp_fft.hip", "slp_fem.hip", "slp_static.hip", "slp_api.cpp", "slp_near.cpp", "slp_fem.cpp",
           "slp_amg.cpp", "slp_server.cpp"]
ARCH = os.environ.get("SLP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libslp)")


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(LIBDIR, src + ".o")
        cmd = [hipcc()] + common
        if src.endswith(".hip"):
            # packed FP32 instructions are disabled for all device code
            cmd += ["-x", "hip", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        cmd += ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
