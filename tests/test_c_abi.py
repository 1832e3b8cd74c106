"""The C ABI driven by a plain C-style program (tests/c/abi_check.cpp, built
by __graft_entry__.build() against the in-tree libbwla.so): device buffers
from hipMalloc, a stream of its own, workspaces sized by the library, no
Python and no torch in the process.  Its inputs are small integers, so every
result it checks has an exact value computed on the host."""
from __future__ import annotations

import os
import subprocess

import pytest

from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c", "abi_check")


def test_plain_c_caller():
    need_gpu()
    assert os.path.exists(EXE), "tests/c/abi_check is built by __graft_entry__.build()"
    p = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0 and "abi check ok" in p.stdout, p.stdout + p.stderr
    assert "FAIL" not in p.stdout
