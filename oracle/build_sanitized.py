"""AddressSanitizer + UndefinedBehaviorSanitizer build of the CPU oracle
(test infrastructure): oracle/sanitize_check.c compiles psc_oracle.c into
one program and runs every entry point the tests use.

    python oracle/build_sanitized.py [n] [threads]
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    out = os.path.join(BUILD, "sanitize_check")
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(HERE, "sanitize_check.c"), "-o", out, "-lm"], check=True)
    return out


def run(n: int = 12, threads: int = 16) -> subprocess.CompletedProcess:
    exe = build()
    e = dict(os.environ, OMP_NUM_THREADS=str(threads), ASAN_OPTIONS="detect_leaks=1:exitcode=66",
             UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return subprocess.run([exe, str(n)], env=e, capture_output=True, text=True)


if __name__ == "__main__":
    r = run(int(sys.argv[1]) if len(sys.argv) > 1 else 12, int(sys.argv[2]) if len(sys.argv) > 2 else 16)
    print(r.stdout + r.stderr)
    sys.exit(r.returncode)
