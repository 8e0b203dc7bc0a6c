"""Build the HIP library ``libgp.so`` in-tree for gfx950 (MI355X).

Every translation unit is compiled with ``-ffp-contract=off`` (FP64 expressions are
evaluated exactly as written, never fused) and with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgp.so")
SOURCES = ["gp_kernels.hip", "gp_serve.hip", "gp_probe.hip", "gp_noalloc.hip", "gp_api.cpp"]
ARCH = os.environ.get("GP_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXXFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *CXXFLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{msg}")
    if msg.strip():
        print(msg, file=sys.stderr)
    return obj


CPU_SRC = os.path.join(HERE, "cpu", "gp_cpu.cpp")
CPU_LIB = os.path.join(HERE, "libgp_cpu.so")
CPU_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-Wall", "-Wextra"]


def build_cpu(verbose: bool = False) -> str:
    """The host SIMD/multi-core implementation (libgp_cpu.so).  Its AVX-512 functions
    carry their own target attribute, so the library runs, scalar, on any x86-64."""
    tmp = CPU_LIB + ".tmp"
    r = subprocess.run(["g++", *CPU_FLAGS, CPU_SRC, "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build of libgp_cpu.so failed:\n" + r.stdout + r.stderr)
    if (r.stdout + r.stderr).strip():
        print(r.stdout + r.stderr, file=sys.stderr)
    os.replace(tmp, CPU_LIB)
    if verbose:
        print("built", CPU_LIB)
    return CPU_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link of libgp.so failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    build_cpu(verbose=True)
