"""Scheduling core of the serving engine, on the CPU under ThreadSanitizer and
AddressSanitizer.

Builds tests/cpp/engine_core_test.cpp (host code only, no HIP, no cipher)
and runs it: budget, FIFO admission, ticket lifecycle, timeouts, rejection
and shutdown with several submitting threads.  The ThreadSanitizer build uses
LLVM's clang++ from the ROCm toolchain: GCC 11's sanitizer runtime does not
intercept pthread_cond_clockwait (used by std::condition_variable with the
steady clock) and reports a false "double lock".
"""
from __future__ import annotations

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.parametrize("sanitize", ["thread", "address", None])
def test_engine_core(tmp_path, sanitize):
    exe = tmp_path / "engine_core_test"
    src = os.path.join(HERE, "cpp", "engine_core_test.cpp")
    if sanitize:
        if not os.path.exists(CLANG):
            pytest.skip("LLVM clang++ not found")
        cmd = [CLANG, f"-fsanitize={sanitize}", "-std=c++17", "-O1", "-g", "-pthread", "-o", str(exe), src]
    else:
        cmd = ["g++", "-std=c++17", "-O2", "-g", "-pthread", "-o", str(exe), src]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "engine core ok" in res.stdout
