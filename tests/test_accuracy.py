"""Accuracy report of the reductions against the float64 oracle, for every
storage type and accumulation mode (run with -s to see the table).  Errors are
stated two ways:

* vs the oracle on the stored (quantised) inputs -- the accumulation error the
  kernels add, held to 1e-12 (f64) and 1e-5 (f32, bf16);
* vs the exact dot of the unquantised float64 draws -- the end-to-end error,
  dominated by rounding the inputs to the storage type (reported, not bounded).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.criteria import TOL, check_scalar, check_vector
from tests.gpu_util import host, need_gpu

pytestmark = pytest.mark.gpu

ROWS = []


@pytest.mark.parametrize("dist", ["uniform", "normal"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_dot_accuracy(dtype, dist):
    need_gpu()
    from paper_1409_0669_amd import ops
    n = 1 << 22
    a = W.draw(dist, n, 0, 31)
    b = W.draw(dist, n, 0, 32)
    sa, sb = W.quantize(a, dtype), W.quantize(b, dtype)
    xa, xb = W.widen(sa, dtype), W.widen(sb, dtype)
    ta, tb = W.to_torch(sa, dtype), W.to_torch(sb, dtype)
    ref_q = oracle.dot(xa, xb)
    ref_full = oracle.dot(a, b)
    for acc in ("plain", "compensated"):
        for od in ((torch.float64,) if dtype == "f64" else (torch.float32, torch.float64)):
            got = float(ops.dot(ta, tb, acc=acc, out_dtype=od).item())
            check_scalar(got, ref_q, 0.0, TOL[dtype], "%s %s %s" % (dtype, acc, od))
            ROWS.append(("dot", dtype, dist, acc, str(od).split(".")[-1], abs(got - ref_q) / abs(ref_q),
                         abs(got - ref_full) / abs(ref_full)))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_gemv_accuracy(dtype):
    need_gpu()
    from paper_1409_0669_amd import ops
    m = n = 2048
    a = W.uniform(m * n, 0, 33).reshape(m, n)
    x = W.uniform(n, 0, 34)
    sa, sx = W.quantize(a, dtype), W.quantize(x, dtype)
    A64, x64 = W.widen(sa, dtype), W.widen(sx, dtype)
    ref_q = oracle.gemv(A64, x64)
    ref_full = oracle.gemv(a, x)
    scale = np.abs(A64) @ np.abs(x64)
    tA, tx = W.to_torch(sa, dtype).reshape(m, n), W.to_torch(sx, dtype)
    for acc in ("plain", "compensated"):
        got = host(ops.gemv(tA, tx, acc=acc, out_dtype=torch.float64))
        check_vector(got, ref_q, scale, TOL[dtype], "%s %s" % (dtype, acc))
        ROWS.append(("gemv", dtype, "uniform", acc, "float64", float(np.max(np.abs(got - ref_q) / scale)),
                     float(np.max(np.abs(got - ref_full) / (np.abs(a) @ np.abs(x))))))


def test_print_accuracy_table():
    if not ROWS:
        pytest.skip("no rows collected")
    print("\nop    storage dist     acc          out      err_vs_oracle(quantised)  err_vs_fp64_draws")
    for r in ROWS:
        print("%-5s %-7s %-8s %-12s %-8s %.3e                 %.3e" % r)
