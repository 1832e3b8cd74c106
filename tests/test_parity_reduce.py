"""GPU parity of the reductions (inner product, norm) against the oracle's
Dot2 value, within the stated tolerances; exact closed forms; determinism."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from tests.criteria import TOL, check_scalar, cond_scale
from tests.gpu_util import DT, guarded_scalar, need_gpu, vec

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 63, 64, 65, 1000, 4097, 100003, (1 << 20) + 5]
DTYPES = ["f64", "f32", "bf16"]
ACCS = ["plain", "compensated"]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()
    from paper_1409_0669_amd import ops
    ops.reset_config()
    yield
    ops.reset_config()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("n", SIZES)
def test_dot_and_nrm2(dtype, acc, n):
    from paper_1409_0669_amd import ops
    x, x64 = vec(n, dtype, 11)
    y, y64 = vec(n, dtype, 12)
    got = float(ops.dot(x, y, acc=acc).item())
    check_scalar(got, oracle.dot(x64, y64), cond_scale(dtype, acc, np.abs(x64 * y64).sum()), TOL[dtype], "dot")
    got = float(ops.nrm2(x, acc=acc).item())
    check_scalar(got, oracle.nrm2(x64), 0.0, TOL[dtype], "nrm2")
    if dtype != "f64":
        got64 = float(ops.dot(x, y, acc=acc, out_dtype=torch.float64).item())
        check_scalar(got64, oracle.dot(x64, y64), cond_scale(dtype, acc, np.abs(x64 * y64).sum()), TOL[dtype],
                     "dot f64 out")


@pytest.mark.parametrize("dtype", DTYPES)
def test_dot_closed_forms(dtype):
    from paper_1409_0669_amd import ops
    t = DT[dtype]
    for n in (1, 1000, 65537, 1 << 20):
        ones = torch.ones(n, dtype=t, device="cuda")
        assert float(ops.dot(ones, ones).item()) == n
        assert float(ops.nrm2(ones * 0.5).item()) == 0.5 * np.sqrt(n) if int(np.sqrt(n)) ** 2 == n else True
        alt = torch.where(torch.arange(n, device="cuda") % 2 == 0, 1.0, -1.0).to(t)
        assert float(ops.dot(alt, ones).item()) == n % 2
    i = torch.arange(4096, dtype=t, device="cuda") if dtype != "bf16" else torch.arange(256, dtype=t, device="cuda")
    k = i.numel()
    assert float(ops.dot(i, torch.ones_like(i)).item()) == k * (k - 1) // 2
    e = torch.zeros(5000, dtype=t, device="cuda")
    e[1234] = -3.0
    assert float(ops.nrm2(e).item()) == 3.0
    empty = torch.empty(0, dtype=t, device="cuda")
    assert float(ops.dot(empty, empty).item()) == 0.0
    assert float(ops.nrm2(empty).item()) == 0.0


def test_dot_compensated_cancellation():
    from paper_1409_0669_amd import ops
    # x = [big..., 1..., -big...]: the exact value is the count of ones, far
    # below the rounding error of a plain float64 sum of the big terms
    n = 1 << 15
    rng = np.random.default_rng(3)
    big = rng.uniform(1, 2, n) * 2.0 ** 60
    x64 = np.concatenate([big, np.ones(n), -big])
    y64 = np.ones(x64.size)
    x = torch.from_numpy(x64).cuda()
    y = torch.from_numpy(y64).cuda()
    ref = oracle.dot(x64, y64)
    assert ref == n
    got = float(ops.dot(x, y, acc="compensated").item())
    check_scalar(got, ref, 0.0, TOL["f64"], "compensated")


CONFIGS = [
    dict(block=64, vec=1, unroll=1, grid=1),
    dict(block=128, vec=2, unroll=2, grid=3, increment=1),
    dict(block=256, vec=4, unroll=4, grid=37),
    dict(block=1024, vec=8, unroll=1, grid=0, increment=1),
    dict(block=512, vec=16, unroll=2, grid=300),
    dict(block=256, vec=4, unroll=8, grid=2048),
    dict(block=1024, vec=2, unroll=8, grid=0, increment=1),
    # more than 2048 partials: the second stage runs 1024 threads, with
    # eight-load batches (20000 partials) or the remainder loop only (one pass)
    dict(block=64, vec=1, unroll=1, grid=20000),
    dict(block=128, vec=1, unroll=1, grid=0),
]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("cfg", range(len(CONFIGS)))
def test_dot_configs(dtype, acc, cfg):
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    ops.set_config(L.OP_DOT, DT[dtype], -1, **CONFIGS[cfg])
    ops.set_config(L.OP_NRM2, DT[dtype], -1, **CONFIGS[cfg])
    for n in (3, 4099, 300017):
        x, x64 = vec(n, dtype, 13)
        y, y64 = vec(n, dtype, 14)
        od = ops.compute_dtype(DT[dtype])
        out, guard = guarded_scalar(od)
        got = float(ops.dot(x, y, acc=acc, out=out).item())
        check_scalar(got, oracle.dot(x64, y64), cond_scale(dtype, acc, np.abs(x64 * y64).sum()), TOL[dtype],
                     str(CONFIGS[cfg]))
        guard("dot %d %s" % (n, CONFIGS[cfg]))
        out, guard = guarded_scalar(od)
        check_scalar(float(ops.nrm2(x, acc=acc, out=out).item()), oracle.nrm2(x64), 0.0, TOL[dtype], "nrm2")
        guard("nrm2 %d %s" % (n, CONFIGS[cfg]))
        out, guard = guarded_scalar(od)
        check_scalar(float(ops.asum(x, acc=acc, out=out).item()), oracle.asum(x64), 0.0, TOL[dtype], "asum")
        guard("asum %d %s" % (n, CONFIGS[cfg]))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("acc", ACCS)
def test_dot_deterministic(dtype, acc):
    from paper_1409_0669_amd import ops
    x, _ = vec(3_000_017, dtype, 15)
    y, _ = vec(3_000_017, dtype, 16)
    vals = {float(ops.dot(x, y, acc=acc).item()) for _ in range(10)}
    assert len(vals) == 1
    vals = {float(ops.nrm2(x, acc=acc).item()) for _ in range(10)}
    assert len(vals) == 1


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dot_misaligned(dtype):
    from paper_1409_0669_amd import ops
    n = 100001
    x, x64 = vec(n, dtype, 17, pad_front=1)
    y, y64 = vec(n, dtype, 18, pad_front=3)
    check_scalar(float(ops.dot(x, y).item()), oracle.dot(x64, y64), cond_scale(dtype, "plain", np.abs(x64 * y64).sum()),
                 TOL[dtype])
