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

SOURCES = ["assemble.cpp", "plan.cpp", "api.cpp", "serve.cpp", "device.hip", "batch.hip", "stream.hip"]

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


# Host-side checks: the host sources with AddressSanitizer and
# UndefinedBehaviorSanitizer (g++), linked with the device objects of the last
# build(). Nothing on the GPU is instrumented; the library serves host-only
# calls (assembly, validation, planning) run under LD_PRELOAD of libasan.
SAN_LIB = os.path.join(HERE, "_build", "libldopf_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def build_sanitized(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    dev_objs = [os.path.join(objdir, s + ".o") for s in SOURCES if s.endswith(".hip")]
    missing = [o for o in dev_objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"device objects missing ({missing}): run build() first")
    gxx = shutil.which("g++") or "g++"
    host_flags = [f for f in CXX_FLAGS if f != "-O3"] + SAN_FLAGS
    objs = []
    for src in SOURCES:
        if src.endswith(".hip"):
            continue
        obj = os.path.join(objdir, src + ".san.o")
        cmd = [gxx, *host_flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    cmd = [gxx, "-shared", "-o", SAN_LIB, *objs, *dev_objs, "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib", *SAN_FLAGS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
