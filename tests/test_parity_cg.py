"""The fused CG-style update equals the separate scaled additions bitwise and
its inner product matches the oracle within tolerance."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from tests.criteria import TOL, bitwise_equal, check_scalar
from tests.gpu_util import host, need_gpu, vec

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [1, 65, 4097, 1_000_003])
def test_cg_update(dtype, n):
    need_gpu()
    from paper_1409_0669_amd import ops
    x, x64 = vec(n, dtype, 41, dist="normal")
    p, p64 = vec(n, dtype, 42, dist="normal")
    r, r64 = vec(n, dtype, 43, dist="normal")
    q, q64 = vec(n, dtype, 44, dist="normal")
    a = 0.123456789
    rr = float(ops.cg_update(a, x, p, r, q).item())
    ae = oracle.scalar(dtype, a)
    xr = oracle.axpby(dtype, ae, p64, 1.0, x64)
    rref = oracle.axpby(dtype, -ae, q64, 1.0, r64)
    assert bitwise_equal(host(x), xr)
    assert bitwise_equal(host(r), rref)
    check_scalar(rr, oracle.dot(rref, rref), 0.0, TOL[dtype], "rr")
