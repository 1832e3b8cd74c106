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


CG_CONFIGS = [dict(block=64, vec=1, unroll=1, grid=1), dict(block=256, vec=2, unroll=2, grid=7, increment=1),
              dict(block=1024, vec=4, unroll=4, grid=0), dict(block=128, vec=8, unroll=1, grid=300)]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("cfg", range(len(CG_CONFIGS)))
def test_cg_update_configs(dtype, cfg):
    need_gpu()
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    from tests.gpu_util import DT
    ops.reset_config()
    ops.set_config(L.OP_CG, DT[dtype], -1, **CG_CONFIGS[cfg])
    try:
        for n in (3, 4099, 300017):
            x, x64 = vec(n, dtype, 45)
            p, p64 = vec(n, dtype, 46)
            r, r64 = vec(n, dtype, 47)
            q, q64 = vec(n, dtype, 48)
            rr = float(ops.cg_update(-0.3, x, p, r, q, acc="compensated").item())
            ae = oracle.scalar(dtype, -0.3)
            assert bitwise_equal(host(x), oracle.axpby(dtype, ae, p64, 1.0, x64))
            rref = oracle.axpby(dtype, -ae, q64, 1.0, r64)
            assert bitwise_equal(host(r), rref)
            check_scalar(rr, oracle.dot(rref, rref), 0.0, TOL[dtype], str(CG_CONFIGS[cfg]))
    finally:
        ops.reset_config()
