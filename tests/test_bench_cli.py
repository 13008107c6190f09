"""bench.py's command line on the CPU: more than one GPU is refused with a
JSON error line before any device work, and the help text lists the legs'
switches."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU only" in line["error"]


def test_help_lists_the_legs():
    r = run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--sweep", "--no-batch", "--no-serve", "--no-hash", "--no-cpu"):
        assert flag in r.stdout, flag
