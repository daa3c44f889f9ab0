"""AddressSanitizer and UndefinedBehaviorSanitizer builds of host code, run on the CPU.

* the oracle (oracle/oracle.c) under a driver that calls every entry point on
  small seeded graphs for k = 2..8 and all three rootings, and the sparse
  k <= 16 oracle (oracle/oracle16.c) for k = 2..12 (tests/sanitize/oracle_checks.c);
* the library's host runtime: the treelet algebra and per-k lookup tables of
  treelets.cpp with every index the kernels take from them checked against
  the staging layout, the serving arena's first-fit allocator under random
  admission and release, the allocator hooks, and the combine's exact small
  division (tests/sanitize/host_checks.cpp).

Both are compiled with gcc / g++ (host code only; the GPU kernels are not
built here) and must exit 0 with no sanitizer report.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, exe):
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    out = _run(["gcc", "-std=gnu11", *SAN, os.path.join(ROOT, "tests", "sanitize", "oracle_checks.c"),
                os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "oracle16.c"), "-o", exe], exe)
    assert "oracle checks done" in out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists("/opt/rocm/lib/libamdhip64.so"),
                    reason="g++ or the HIP runtime library not available")
def test_host_runtime_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    out = _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"),
                os.path.join(ROOT, "paper_2009_03052_amd", "csrc", "treelets.cpp"),
                "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe], exe)
    assert "host checks done" in out
