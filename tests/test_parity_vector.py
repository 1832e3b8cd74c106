"""GPU parity of the streaming kernels: copy and scaled vector addition are
single-rounding operations, so they must match the oracle bitwise (0 ULP in
matching precision) for every size, alignment, aliasing and configuration."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from tests.criteria import bitwise_equal
from tests.gpu_util import DT, guarded, host, need_gpu, vec

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 7, 63, 64, 65, 255, 1000, 4097, (1 << 20) + 3]
DTYPES = ["f64", "f32", "bf16"]
ALPHA, BETA = 0.7312345678901234, -1.2345678901234567


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()
    from paper_1409_0669_amd import ops
    ops.reset_config()
    yield
    ops.reset_config()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", SIZES)
def test_copy_bitwise(dtype, n):
    from paper_1409_0669_amd import ops
    y, y64 = vec(n, dtype, 1)
    x, guard = guarded(n, dtype)
    ops.copy(y, out=x)
    assert bitwise_equal(host(x), oracle.copy(y64))
    guard("copy")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", SIZES)
def test_axpby_bitwise(dtype, n):
    from paper_1409_0669_amd import ops
    y, y64 = vec(n, dtype, 1)
    z, z64 = vec(n, dtype, 2)
    x, guard = guarded(n, dtype)
    ops.axpby(ALPHA, y, BETA, z, out=x)
    ref = oracle.axpby(dtype, oracle.scalar(dtype, ALPHA), y64, oracle.scalar(dtype, BETA), z64)
    assert bitwise_equal(host(x), ref)
    guard("axpby")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("offsets", [(1, 0, 0), (0, 1, 3), (3, 3, 3)])
def test_axpby_misaligned(dtype, offsets):
    from paper_1409_0669_amd import ops
    n = 10007
    y, y64 = vec(n, dtype, 3, pad_front=offsets[0])
    z, z64 = vec(n, dtype, 4, pad_front=offsets[1])
    out, guard = guarded(n, dtype, offset=offsets[2])
    ops.axpby(ALPHA, y, BETA, z, out=out)
    ref = oracle.axpby(dtype, oracle.scalar(dtype, ALPHA), y64, oracle.scalar(dtype, BETA), z64)
    assert bitwise_equal(host(out), ref)
    guard("misaligned axpby")


@pytest.mark.parametrize("dtype", DTYPES)
def test_axpby_in_place_and_device_scalars(dtype):
    from paper_1409_0669_amd import ops
    n = 70001
    y, y64 = vec(n, dtype, 5)
    z, z64 = vec(n, dtype, 6)
    cd = ops.compute_dtype(DT[dtype])
    a_dev = torch.tensor([0.377], dtype=cd, device="cuda")
    b_dev = torch.tensor([-2.5], dtype=cd, device="cuda")
    a_val, b_val = float(a_dev.item()), float(b_dev.item())
    # x += a*p form: out aliases z
    ops.axpby(0.9, y, 1.0, z, out=z, alpha_dev=a_dev)
    ref = oracle.axpby(dtype, oracle.scalar(dtype, 0.9, a_val), y64, 1.0, z64)
    assert bitwise_equal(host(z), ref)
    # out aliases y, both factors on the device
    ops.axpby(1.5, y, 0.25, z, out=y, alpha_dev=a_dev, beta_dev=b_dev)
    ref2 = oracle.axpby(dtype, oracle.scalar(dtype, 1.5, a_val), y64, oracle.scalar(dtype, 0.25, b_val), ref)
    assert bitwise_equal(host(y), ref2)


CONFIGS = [
    dict(block=64, vec=1, unroll=1, grid=1),
    dict(block=128, vec=2, unroll=2, grid=3, increment=1),
    dict(block=256, vec=4, unroll=4, grid=7),
    dict(block=1024, vec=8, unroll=1, grid=0, increment=1),
    dict(block=512, vec=16, unroll=2, grid=5),
    dict(block=256, vec=16, unroll=4, grid=0),
]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("cfg", range(len(CONFIGS)))
def test_stream_configs_bitwise(dtype, cfg):
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    ops.set_config(L.OP_AXPBY, DT[dtype], -1, **CONFIGS[cfg])
    ops.set_config(L.OP_COPY, DT[dtype], -1, **CONFIGS[cfg])
    for n in (5, 4099, 300017):
        y, y64 = vec(n, dtype, 7)
        z, z64 = vec(n, dtype, 8)
        x, guard = guarded(n, dtype)
        ops.axpby(ALPHA, y, BETA, z, out=x)
        ref = oracle.axpby(dtype, oracle.scalar(dtype, ALPHA), y64, oracle.scalar(dtype, BETA), z64)
        assert bitwise_equal(host(x), ref), (n, CONFIGS[cfg])
        guard("axpby %d %s" % (n, CONFIGS[cfg]))
        c, guard = guarded(n, dtype)
        ops.copy(y, out=c)
        assert bitwise_equal(host(c), y64)
        guard("copy %d %s" % (n, CONFIGS[cfg]))


def test_axpby_empty_and_specials():
    from paper_1409_0669_amd import ops
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    assert ops.axpby(1.0, e, 1.0, e).numel() == 0
    y = torch.tensor([1.0, float("inf"), float("nan"), -0.0, 3.0], dtype=torch.float64, device="cuda")
    z = torch.tensor([float("inf"), 1.0, 1.0, 0.0, -3.0], dtype=torch.float64, device="cuda")
    x = host(ops.axpby(2.0, y, 0.0, z))     # beta = 0 still reads z: 0*inf = nan
    ref = oracle.axpby("f64", 2.0, host(y), 0.0, host(z))
    assert bitwise_equal(x, ref)
    assert np.isnan(x[0])


def test_axpby_and_dot_beyond_2_pow_31_elements():
    """Indices past 2^31: bf16 vectors of 2^31 + 37 elements (4 GiB each),
    axpby checked bitwise on sampled indices (including the tail), and the
    reductions over every element against closed forms."""
    import workloads as W
    from paper_1409_0669_amd import ops
    n = (1 << 31) + 37
    y = W.device_draw(n, "bf16", 0, 70)
    z = W.device_draw(n, "bf16", 0, 71)
    x = ops.axpby(ALPHA, y, BETA, z)
    idx = np.concatenate([np.arange(8), np.random.default_rng(0).integers(0, n, 4096), np.arange(n - 64, n)])
    ti = torch.from_numpy(idx).cuda()
    y64, z64, x64 = host(y[ti]), host(z[ti]), host(x[ti])
    ref = oracle.axpby("bf16", oracle.scalar("bf16", ALPHA), y64, oracle.scalar("bf16", BETA), z64)
    assert bitwise_equal(x64, ref)
    del x, y, z
    # the reductions over all 2^31 + 37 elements: a closed form (every
    # per-thread partial is an exactly representable count)
    ones = torch.ones(n, dtype=torch.bfloat16, device="cuda")
    assert float(ops.dot(ones, ones, out_dtype=torch.float64).item()) == n
    assert float(ops.dot(ones, ones, acc="compensated", out_dtype=torch.float64).item()) == n
    nr = float(ops.nrm2(ones, out_dtype=torch.float64).item())
    assert abs(nr - np.sqrt(n)) <= 1e-12 * np.sqrt(n)
