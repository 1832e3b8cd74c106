"""BWLA_LOG: with it set, every call that launches kernels writes one line to
stderr naming the entry point, storage type, accumulation mode, kernel shape
and the resolved configuration; calls that fail validation or have nothing to
do write nothing."""
from __future__ import annotations

import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LINE = re.compile(r"^bwla: (?P<what>[a-z_0-9 ]+?) (?P<dtype>f64|f32|bf16) (?P<acc>plain|compensated|-) "
                  r"m=(?P<m>\d+) n=(?P<n>\d+) block=(?P<block>\d+) vec=(?P<vec>\d+) unroll=(?P<unroll>\d+) "
                  r"grid=(?P<grid>\d+) increment=(?P<increment>\d+) rows=(?P<rows>\d+) split=(?P<split>\d+)$")
FIELDS = ("block", "vec", "unroll", "grid", "increment", "rows", "split")


def _child(code: str, log: str = "1"):
    env = dict(os.environ, BWLA_LOG=log, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, text=True, timeout=300)
    assert p.returncode == 0, p.stderr[-3000:]
    return p.stdout, p.stderr


def test_no_line_without_a_launch():
    code = ("from paper_1409_0669_amd import _lib as L\n"
            "F = 1 << 40\n"
            "assert L.lib.bwla_copy(0, -1, F, F + 4096, None) == L.ERR_INVALID_ARG\n"
            "assert L.lib.bwla_copy(0, 0, None, None, None) == L.OK\n"
            "assert L.lib.bwla_axpby(7, 10, 1.0, None, F, 1.0, None, F + 4096, F + 8192, None) == L.ERR_UNSUPPORTED\n")
    _, err = _child(code)
    assert "bwla:" not in err


@pytest.mark.gpu
def test_each_launch_logs_its_resolved_configuration():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    code = r'''
import json, torch
from paper_1409_0669_amd import ops, _lib as L
ops.reset_config()
assert ops.load_default_tuning()
n = 1 << 20
x = torch.rand(n, dtype=torch.float64, device="cuda")
y = torch.rand(n, dtype=torch.float64, device="cuda")
A = torch.rand(4096, 1024, dtype=torch.float32, device="cuda")
u = torch.rand(1024, dtype=torch.float32, device="cuda")
w = torch.rand(4096, dtype=torch.float32, device="cuda")
ops.axpby(0.5, x, 2.0, y)
ops.dot(x, y)
ops.dot(x, y, acc="compensated")
ops.nrm2(x)
ops.gemv(A, u)
ops.gemv(A, w, trans=True, acc="compensated")
torch.cuda.synchronize()
exp = [
    ("axpby", "f64", "-", 1, n, ops.get_config(L.OP_AXPBY, torch.float64, 0, n)),
    ("dot", "f64", "plain", 1, n, ops.get_config(L.OP_DOT, torch.float64, 0, n)),
    ("dot", "f64", "compensated", 1, n, ops.get_config(L.OP_DOT, torch.float64, 0, n, acc="compensated")),
    ("nrm2", "f64", "plain", 1, n, ops.get_config(L.OP_NRM2, torch.float64, 0, n)),
    ("gemv rows", "f32", "plain", 4096, 1024, ops.get_config(L.OP_GEMV_ROWS, torch.float32, 4096, 1024)),
    ("gemv cols", "f32", "compensated", 4096, 1024,
     ops.get_config(L.OP_GEMV_COLS, torch.float32, 4096, 1024, acc="compensated")),
]
print(json.dumps(exp))
'''
    out, err = _child(code)
    lines = [l for l in err.splitlines() if l.startswith("bwla:")]
    exp = json.loads(out.strip().splitlines()[-1])
    assert len(lines) == len(exp), err
    for line, (what, dtype, acc, m, n, cfg) in zip(lines, exp):
        g = LINE.match(line)
        assert g, line
        assert (g["what"], g["dtype"], g["acc"], int(g["m"]), int(g["n"])) == (what, dtype, acc, m, n), line
        assert {k: int(g[k]) for k in FIELDS} == {k: int(cfg[k]) for k in FIELDS}, (line, cfg)
    out, err = _child(code, log="0")
    assert "bwla:" not in err
