"""One HIP runtime per process, whatever the import order.

PyTorch's wheels ship their own libamdhip64 / libhsa-runtime64 and ask for
them under a different file name than libaesctr.so does; if the library
loaded first, with ROCm's copies, the process would end up with two HIP
runtimes whose streams and devices do not mix.  The binding loads PyTorch
first.  Loading shared libraries needs no GPU, so this runs on the CPU.
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = """
import {first}, {second}
libs = sorted({{l.split()[-1] for l in open('/proc/self/maps')
              if 'libamdhip64' in l or 'libhsa-runtime64' in l}})
print(len([p for p in libs if 'libamdhip64' in p]), len([p for p in libs if 'libhsa-runtime64' in p]))
"""


@pytest.mark.parametrize("order", [("paper_2607_02630_amd", "torch"), ("torch", "paper_2607_02630_amd"),
                                   ("paper_2607_02630_amd.loadgen", "torch")])
def test_single_hip_runtime(order):
    code = PROBE.format(first=order[0], second=order[1])
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert res.returncode == 0, res.stderr
    assert res.stdout.split() == ["1", "1"], res.stdout
