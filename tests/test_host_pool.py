"""Host thread pool of the library (validation and staging of large batches),
on the CPU under ThreadSanitizer, AddressSanitizer and neither.

Builds tests/cpp/host_pool_test.cpp together with the library's own
csrc/host_pool.cpp (host code only, no HIP) and runs it: every index of a
parallel_for runs once, parts are the documented ranges, and concurrent
callers and thousands of back-to-back jobs lose no work.  The sanitizer
build uses LLVM's clang++ from the ROCm toolchain (see test_engine_core.py).
"""
from __future__ import annotations

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
POOL = os.path.join(HERE, "..", "paper_2607_02630_amd", "csrc", "host_pool.cpp")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.parametrize("sanitize", ["thread", "address", None])
def test_host_pool(tmp_path, sanitize):
    exe = tmp_path / "host_pool_test"
    src = os.path.join(HERE, "cpp", "host_pool_test.cpp")
    if sanitize:
        if not os.path.exists(CLANG):
            pytest.skip("LLVM clang++ not found")
        cmd = [CLANG, f"-fsanitize={sanitize}", "-std=c++17", "-O1", "-g", "-pthread", "-o", str(exe), src, POOL]
    else:
        cmd = ["g++", "-std=c++17", "-O2", "-g", "-pthread", "-o", str(exe), src, POOL]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "host pool ok" in res.stdout
