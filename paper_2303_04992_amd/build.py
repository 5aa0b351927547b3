"""Build libkfbi.so in-tree for gfx950 (hipcc; host setup with OpenMP).

Usage: python paper_2303_04992_amd/build.py   (or __graft_entry__.build())
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libkfbi.so")

HIP_SOURCES = ["kernels.hip", "gemm.hip", "api.hip"]
CPP_SOURCES = ["geometry.cpp", "surface.cpp", "assemble.cpp"]

ARCH = os.environ.get("KFBI_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
# packed fp32 instructions stay off (plain scalar fp32 code only)
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(OUT, s + ".o")
        jobs.append([hipcc(), *COMMON, *HIP_FLAGS, "-c", os.path.join(SRC, s), "-o", o])
        objs.append(o)
    for s in CPP_SOURCES:
        o = os.path.join(OUT, s + ".o")
        jobs.append(["g++", *COMMON, "-march=x86-64-v2", "-fopenmp", "-c", os.path.join(SRC, s), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr, file=sys.stderr)
    tmp = LIB + ".tmp"
    _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lgomp"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
