"""Build libldopf.so in place with hipcc for gfx950.

Usage: python -m paper_2310_09410_amd.build  (or call ``build()``).
Every call recompiles; the shared library lands next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libldopf.so")
ARCH = "gfx950"

SOURCES = ["assemble.cpp", "plan.cpp", "api.cpp", "serve.cpp", "device.hip", "batch.hip"]

# -packed-fp32-ops keeps the compiler from emitting packed FP32 arithmetic.
HIP_FLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
# Host-only sources (assembly, planning, the C ABI, the serving runtime) hold
# no device code: plain C++ against the HIP runtime headers.
CXX_FLAGS = [
    "-x", "c++", "-D__HIP_PLATFORM_AMD__=1", "-isystem", "/opt/rocm/include",
    "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    cand = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cand):
        raise RuntimeError("hipcc not found")
    return cand


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        flags = HIP_FLAGS if src.endswith(".hip") else CXX_FLAGS
        cmd = [hipcc(), *flags, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
