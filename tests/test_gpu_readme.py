"""The README's usage example runs as written and its outputs decrypt back
(GPU)."""
from __future__ import annotations

import os
import re

import pytest

from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_usage_example():
    torch = torch_cuda()
    text = open(os.path.join(ROOT, "README.md")).read()
    code = re.search(r"## Use\s+```python\n(.*?)```", text, re.S).group(1)
    scope: dict = {}
    exec(compile(code, "README.md", "exec"), scope)
    torch.cuda.synchronize()
    A, s, x, y, z = scope["A"], scope["s"], scope["x"], scope["y"], scope["z"]
    # y = x under counter 1 (single call), z = x under counter 7 (engine):
    # decrypting each with its own counter gives x back, and they differ.
    assert torch.equal(A.aes_ctr_crypt(s, bytes(12), 1, y), x)
    assert torch.equal(A.aes_ctr_crypt(s, bytes(12), 7, z), x)
    assert not torch.equal(y, z)
