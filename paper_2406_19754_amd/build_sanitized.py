"""CPU sanitizer builds of the library's host-side setup code (not part of
libpsc.so): csrc/host_check.cpp drives setup.cpp and fai.cpp through the
build sequence of one process building several hierarchies (see that file),
with the GPU coarsening stubbed so every level takes the host path.

  asan  g++, AddressSanitizer + UndefinedBehaviorSanitizer, libgomp
  tsan  clang++ (the ROCm LLVM), ThreadSanitizer with the LLVM OpenMP
        runtime and its Archer tool, which tells TSan about OpenMP's
        barriers and tasks (libgomp is not instrumented: TSan reports its
        synchronisation as races)

    python paper_2406_19754_amd/build_sanitized.py [asan|tsan] [n] [threads]
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LLVM = "/opt/rocm/llvm"
SOURCES = [os.path.join(CSRC, f) for f in ("setup.cpp", "fai.cpp", "host_check.cpp")]


def build(kind: str = "asan") -> str:
    os.makedirs(BUILD, exist_ok=True)
    out = os.path.join(BUILD, f"host_check_{kind}")
    common = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-I", INCLUDE]
    if kind == "asan":
        cmd = ["g++"] + common + ["-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    elif kind == "tsan":
        cmd = [os.path.join(LLVM, "bin", "clang++")] + common + [
            "-fopenmp", "-fsanitize=thread", f"-Wl,-rpath,{os.path.join(LLVM, 'lib')}"]
    else:
        raise ValueError(kind)
    subprocess.run(cmd + SOURCES + ["-o", out], check=True)
    return out


def env(kind: str, threads: int) -> dict:
    e = dict(os.environ, OMP_NUM_THREADS=str(threads))
    if kind == "asan":
        e["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=66"
        e["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    else:
        e["OMP_TOOL_LIBRARIES"] = os.path.join(LLVM, "lib", "libarcher.so")
        e["TSAN_OPTIONS"] = "ignore_noninstrumented_modules=1:exitcode=66"
    return e


def run(kind: str = "asan", n: int = 24, threads: int = 16, names: str = "") -> subprocess.CompletedProcess:
    exe = build(kind)
    args = [exe, str(n), "1"] + ([names] if names else [])
    return subprocess.run(args, env=env(kind, threads), capture_output=True, text=True)


if __name__ == "__main__":
    k = sys.argv[1] if len(sys.argv) > 1 else "asan"
    r = run(k, int(sys.argv[2]) if len(sys.argv) > 2 else 24, int(sys.argv[3]) if len(sys.argv) > 3 else 16)
    print(r.stdout + r.stderr)
    sys.exit(r.returncode)
