"""Build libcsmap.so in-tree for gfx950.

The HIP sources are compiled with hipcc for gfx950 only, without
floating-point contraction (explicit fma calls in the kernels fix every
fused operation) and with packed FP32 instructions disabled.  The library is
linked against the HIP runtime that PyTorch loads (same SONAME), so a process
that imports torch and libcsmap holds a single HIP runtime.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import sysconfig

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcsmap.so")
ROOT = os.path.dirname(HERE)

HIP_SOURCES = ["kernels.hip", "alm.hip", "flat.hip", "probe.hip", "api.cpp"]
CXX_SOURCES = ["sched.cpp", "cones.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I" + os.path.join(ROOT, "include"),
]


def _torch_lib_dir() -> str | None:
    for base in (sysconfig.get_paths().get("purelib"), sysconfig.get_paths().get("platlib")):
        if base:
            d = os.path.join(base, "torch", "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    return None


def _hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libcsmap")


def build(verbose: bool = False) -> str:
    """Compile every source and link libcsmap.so.  Always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    objs = []

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"build step failed: {' '.join(cmd)}")
        # The host pass does not know the packed-FP32 feature; that warning is harmless.
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l)
        if verbose and msg.strip():
            sys.stderr.write(msg + "\n")

    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        run([hipcc, *HIPCC_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        run(["g++", "-O2", "-fPIC", "-std=c++17", "-Wall", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tl = _torch_lib_dir()
    link = ["g++", "-shared", "-o", LIB + ".tmp", *objs, "-Wl,--no-undefined"]
    rpath = []
    if tl:
        link += ["-L" + tl]
        rpath.append(tl)
    link += ["-L/opt/rocm/lib", "-l:libamdhip64.so"]
    rpath.append("/opt/rocm/lib")
    link += ["-Wl,-rpath," + ":".join(rpath)]
    run(link)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
