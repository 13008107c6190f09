"""Every Python source of the package, the benchmark and the build entry
compiles (a syntax error in a module only the GPU runs would otherwise
surface there first)."""
from __future__ import annotations

import glob
import os
import py_compile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = sorted(glob.glob(os.path.join(ROOT, "paper_2607_02630_amd", "*.py"))
                 + glob.glob(os.path.join(ROOT, "paper_2607_02630_amd", "csrc", "*.py"))
                 + [os.path.join(ROOT, "bench.py"), os.path.join(ROOT, "__graft_entry__.py")])


@pytest.mark.parametrize("path", SOURCES, ids=lambda p: os.path.relpath(p, ROOT))
def test_compiles(path, tmp_path):
    py_compile.compile(path, cfile=str(tmp_path / "out.pyc"), doraise=True)
