"""Scheduling core and key cache of the serving engine, on the CPU under
ThreadSanitizer and AddressSanitizer.

Builds tests/cpp/engine_core_test.cpp (host code only, no HIP, no cipher)
and runs it: budget, FIFO admission, ticket lifecycle, timeouts, rejection
and shutdown with several submitting threads.  tests/cpp/key_cache_test.cpp
drives the resident key cache through random launches against a model of
the device key table (a hit reads a slot holding that key; no slot is
installed into while a launch in flight touches it).  The ThreadSanitizer build uses
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


PROGRAMS = {"engine_core_test": "engine core ok", "key_cache_test": "key cache ok"}


@pytest.mark.parametrize("name", sorted(PROGRAMS))
@pytest.mark.parametrize("sanitize", ["thread", "address", None])
def test_engine_core(tmp_path, sanitize, name):
    exe = tmp_path / name
    src = os.path.join(HERE, "cpp", f"{name}.cpp")
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
    assert PROGRAMS[name] in res.stdout
