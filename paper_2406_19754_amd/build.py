"""Build libpsc.so in-tree: host setup with g++ (OpenMP), kernels with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpsc.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIP_SOURCES = ["amg.hip", "net.hip", "gsetup.hip"]
# device setup reproduces the host setup bit for bit: no contraction there
EXACT_SOURCES = ["gsetup.hip"]
CXX_SOURCES = ["setup.cpp", "fai.cpp"]
HEADERS = ["kernels.h", "setup.h", "net.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are switched off (wrong results were seen from
# some of their forms on this hardware); hipcc's host pass warns harmlessly.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=fast",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-I", INCLUDE]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
             "-Wall", "-I", INCLUDE]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def sources():
    return ([os.path.join(CSRC, s) for s in HIP_SOURCES + CXX_SOURCES + HEADERS]
            + [os.path.join(INCLUDE, "psc.h")])


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source (always) and link libpsc.so."""
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for s in CXX_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmd = ["g++"] + CXX_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(o)
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        flags = HIP_FLAGS
        if s in EXACT_SOURCES:
            flags = [f if f != "-ffp-contract=fast" else "-ffp-contract=off" for f in HIP_FLAGS]
        cmd = [HIPCC] + flags + ["-c", os.path.join(CSRC, s), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(o)
    bad = [p.args for p in procs if p.wait() != 0]
    if bad:
        raise RuntimeError("compilation failed: " + " ".join(bad[0]))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lgomp"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
