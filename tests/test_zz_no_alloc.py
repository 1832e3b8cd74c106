"""The inner product for callers that cannot allocate (bwla_dot_noalloc):
called through the C ABI, it must return bitwise what bwla_dot returns on the
same inputs in the same configuration, on two calls in a row with the second
input smaller, for every storage type and accumulation mode -- also with a
configuration whose first stage fills the whole static scratch (65536
work-groups) followed by a smaller one.  Both are also within the oracle's
criteria."""
from __future__ import annotations

import ctypes

import pytest
import torch

import oracle
from tests.criteria import TOL, bitwise_equal, check_scalar, cond_scale
from tests.gpu_util import DT, need_gpu, vec

pytestmark = pytest.mark.gpu

CODE = {"f64": 0, "f32": 1, "bf16": 2}
OUT = {"f64": 0, "f32": 1, "bf16": 1}


def _pair(L, dtype, acc, n, stream):
    """(bwla_dot result, bwla_dot_noalloc result, x64, y64) on fresh inputs."""
    from paper_1409_0669_amd import ops
    x, x64 = vec(n, dtype, stream)
    y, y64 = vec(n, dtype, stream + 1)
    od = torch.float64 if dtype == "f64" else torch.float32
    a = torch.full((), float("nan"), dtype=od, device="cuda")
    b = torch.full((), float("nan"), dtype=od, device="cuda")
    nbytes = ctypes.c_size_t()
    L.check(L.lib.bwla_workspace_size(L.OP_DOT, CODE[dtype], acc, 0, 0, 0, n, ctypes.byref(nbytes)))
    ws = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device="cuda")
    s = ops._stream()
    L.check(L.lib.bwla_dot(CODE[dtype], acc, n, x.data_ptr(), y.data_ptr(), OUT[dtype], a.data_ptr(),
                           ws.data_ptr(), nbytes.value, s))
    L.check(L.lib.bwla_dot_noalloc(CODE[dtype], acc, n, x.data_ptr(), y.data_ptr(), OUT[dtype], b.data_ptr(), s))
    torch.cuda.synchronize()
    return float(a.item()), float(b.item()), x64, y64


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("acc", [0, 1])
def test_noalloc_equals_dot_on_two_calls(dtype, acc):
    need_gpu()
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    ops.reset_config()
    assert ops.load_default_tuning()
    for n, stream in (((1 << 22) + 3, 1610), (100_003, 1620)):
        a, b, x64, y64 = _pair(L, dtype, acc, n, stream)
        assert bitwise_equal(b, a), (dtype, acc, n, a, b)
        check_scalar(b, oracle.dot(x64, y64), cond_scale(dtype, acc, abs(x64 * y64).sum()), TOL[dtype],
                     "%s acc=%d n=%d" % (dtype, acc, n))
    ops.reset_config()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_full_scratch_then_smaller(dtype):
    """A grid of 65536 work-groups writes every slot of the scratch; the
    next, smaller call (default grid) must not see the stale slots."""
    need_gpu()
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    ops.reset_config()
    try:
        ops.set_config(L.OP_DOT, DT[dtype], -1, block=64, vec=1, unroll=1, grid=65536)
        n = 65536 * 64 + 5
        assert ops.get_config(L.OP_DOT, DT[dtype], 0, n)["grid"] == 65536
        a, b, x64, y64 = _pair(L, dtype, 1, n, 1630)
        assert bitwise_equal(b, a)
        check_scalar(b, oracle.dot(x64, y64), 0.0, TOL[dtype], "full scratch")
        ops.reset_config()
        a, b, x64, y64 = _pair(L, dtype, 1, 40_001, 1640)
        assert bitwise_equal(b, a)
        check_scalar(b, oracle.dot(x64, y64), 0.0, TOL[dtype], "after full scratch")
    finally:
        ops.reset_config()


def test_noalloc_empty_and_binding():
    """n = 0 writes 0; the ops binding calls the same entry point."""
    need_gpu()
    from paper_1409_0669_amd import ops
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    out = torch.full((), 7.0, dtype=torch.float64, device="cuda")
    ops.dot_noalloc(e, e, out=out)
    assert float(out.item()) == 0.0
    x, x64 = vec(5003, "f32", 1650)
    y, y64 = vec(5003, "f32", 1651)
    got = float(ops.dot_noalloc(x, y, acc="compensated").item())
    assert bitwise_equal(got, float(ops.dot(x, y, acc="compensated").item()))
    check_scalar(got, oracle.dot(x64, y64), 0.0, TOL["f32"], "binding")
