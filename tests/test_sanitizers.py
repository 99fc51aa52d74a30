"""Sanitizer runs of the host code on the CPU (no GPU): the library's host
setup and smoother-factor code under AddressSanitizer + UBSan and under
ThreadSanitizer (LLVM OpenMP with its Archer tool), replaying a process that
builds six hierarchies in a row, each packed for upload and rebuilt; and the
oracle under AddressSanitizer + UBSan through every entry point the tests
use. Sixteen OpenMP threads, the thread count of the GPU host's share."""
import os
import shutil

import pytest

pytestmark = pytest.mark.slow


def _check(r, what):
    out = r.stdout + r.stderr
    assert r.returncode == 0, f"{what} exited {r.returncode}:\n{out[-4000:]}"
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]


def test_host_setup_under_asan_ubsan():
    from paper_2406_19754_amd import build_sanitized as B
    r = B.run("asan", n=24, threads=16)
    _check(r, "host_check (ASan + UBSan)")
    assert "host check ok" in r.stdout


@pytest.mark.skipif(not os.path.exists("/opt/rocm/llvm/lib/libarcher.so"), reason="LLVM OpenMP Archer tool missing")
def test_host_setup_under_tsan():
    from paper_2406_19754_amd import build_sanitized as B
    r = B.run("tsan", n=16, threads=16)
    _check(r, "host_check (TSan)")
    assert "host check ok" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_asan_ubsan():
    from oracle import build_sanitized as O
    r = O.run(n=12, threads=16)
    _check(r, "oracle sanitize_check (ASan + UBSan)")
    assert "sanitize check ok" in r.stdout
