"""GPU parity of the GEMV with the inner-product epilogue (y = op(A) x and
<w, y> in one launch sequence) against the oracle's two definitions in
sequence."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from tests.criteria import TOL, bitwise_equal, check_scalar, check_vector, plain_reduced
from tests.gpu_util import DT, host, mat, need_gpu, vec

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 7), (7, 1), (33, 65), (257, 1023), (1000, 3001), (64, 20000), (5000, 40)]
ROWS_CFG = [dict(block=64, vec=1, rows=1, split=1), dict(block=128, vec=2, rows=2, split=3),
            dict(block=256, vec=4, rows=8, split=1), dict(block=1024, vec=4, rows=4, split=2),
            dict(block=512, vec=2, rows=8, split=7)]
COLS_CFG = [dict(block=64, vec=1, unroll=1, split=1), dict(block=128, vec=2, unroll=2, split=3),
            dict(block=256, vec=4, unroll=4, split=1), dict(block=1024, vec=4, unroll=4, split=2),
            dict(block=512, vec=2, unroll=1, split=9)]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()
    from paper_1409_0669_amd import ops
    ops.reset_config()
    yield
    ops.reset_config()


def _check(dtype, acc, A64, x64, w64, trans, y, s, what):
    """y against the oracle's GEMV (componentwise, condition-scaled), and s
    against the oracle's <w, RN(op(A) x)> within
    2 tol sum_i |w_i| (|op(A)| |x|)_i: each stored y_i may differ from the
    oracle's by tol (|op(A)| |x|)_i, and the reduction adds at most
    tol sum |w_i y_i| <= tol sum_i |w_i| (|op(A)| |x|)_i."""
    B = A64.T if trans else A64
    ref_y, ref_s = oracle.gemv_dot(dtype, np.ascontiguousarray(B), x64, w64)
    scale = np.abs(B) @ np.abs(x64)
    check_vector(host(y), ref_y, scale, TOL[dtype], what + " y", plain_f32=plain_reduced(dtype, acc))
    check_scalar(float(s.item()), ref_s, 2.0 * float(np.abs(w64) @ scale), TOL[dtype], what + " s")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["row", "col"])
@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_gemv_dot(dtype, layout, trans, shape):
    from paper_1409_0669_amd import ops
    m, n = shape
    A, A64 = mat(m, n, dtype, 41, layout=layout)
    x, x64 = vec(m if trans else n, dtype, 42)
    w, w64 = vec(n if trans else m, dtype, 43)
    for acc in ("plain", "compensated"):
        y, s = ops.gemv_dot(A, x, w, trans=bool(trans), acc=acc)
        assert y.dtype == DT[dtype] and s.dtype == DT[dtype]
        _check(dtype, acc, A64, x64, w64, trans, y, s, "%s %s t=%d %s %s" % (dtype, layout, trans, shape, acc))
        # y is exactly what the GEMV alone stores (same kernel, same order)
        assert bitwise_equal(host(y), host(ops.gemv(A, x, trans=bool(trans), acc=acc)))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("cfg", range(len(ROWS_CFG)))
def test_gemv_dot_configs(dtype, cfg):
    """Every combination of pack width, rows per work-group and split: the
    epilogue sits in the rows or cols kernel (split 1) or in the line
    combine (split > 1)."""
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    ops.set_config(L.OP_GEMV_ROWS, DT[dtype], -1, **ROWS_CFG[cfg])
    ops.set_config(L.OP_GEMV_COLS, DT[dtype], -1, **COLS_CFG[cfg])
    for (m, n) in [(37, 3000), (2500, 131), (513, 515)]:
        for layout in ("row", "col"):
            A, A64 = mat(m, n, dtype, 44, layout=layout)
            for trans in (0, 1):
                x, x64 = vec(m if trans else n, dtype, 45)
                w, w64 = vec(n if trans else m, dtype, 46)
                for acc in ("plain", "compensated"):
                    y, s = ops.gemv_dot(A, x, w, trans=bool(trans), acc=acc)
                    _check(dtype, acc, A64, x64, w64, trans, y, s, "cfg %d %s t=%d %s" % (cfg, layout, trans, acc))


@pytest.mark.parametrize("layout", ["row", "col"])
def test_gemv_dot_cg_pair_alias_and_f64_dot(layout):
    """The q = A p, <p, q> pair (w aliases x), float32 storage with a float64
    inner product, and a padded leading dimension."""
    from paper_1409_0669_amd import ops
    n = 1537
    A, A64 = mat(n, n, "f32", 47, layout=layout, pad=3)
    p, p64 = vec(n, "f32", 48)
    for acc in ("plain", "compensated"):
        q, s = ops.gemv_dot(A, p, acc=acc, dot_dtype=torch.float64)
        assert s.dtype == torch.float64
        _check("f32", acc, A64, p64, p64, 0, q, s, "cg pair %s %s" % (layout, acc))


def test_gemv_dot_exact_integers():
    """Small integers: every product and partial sum is exact in float64, so
    y and <w, y> are exact whatever the order."""
    from paper_1409_0669_amd import ops
    rng = np.random.default_rng(7)
    m, n = 700, 1300
    A64 = rng.integers(-8, 9, (m, n)).astype(np.float64)
    x64 = rng.integers(-8, 9, n).astype(np.float64)
    w64 = rng.integers(-8, 9, m).astype(np.float64)
    y, s = ops.gemv_dot(torch.from_numpy(A64).cuda(), torch.from_numpy(x64).cuda(), torch.from_numpy(w64).cuda())
    assert bitwise_equal(host(y), A64 @ x64)
    assert float(s.item()) == float(w64 @ (A64 @ x64))


def test_gemv_dot_empty():
    from paper_1409_0669_amd import ops
    s_prev = torch.full((), 5.0, dtype=torch.float64, device="cuda")
    A = torch.zeros(0, 6, dtype=torch.float64, device="cuda")
    y, s = ops.gemv_dot(A, torch.ones(6, dtype=torch.float64, device="cuda"),
                        torch.zeros(0, dtype=torch.float64, device="cuda"), dot_out=s_prev)
    assert y.numel() == 0 and float(s.item()) == 0.0
    A = torch.zeros(4, 0, dtype=torch.float32, device="cuda")
    y = torch.full((4,), 3.0, dtype=torch.float32, device="cuda")
    y, s = ops.gemv_dot(A, torch.zeros(0, dtype=torch.float32, device="cuda"),
                        torch.ones(4, dtype=torch.float32, device="cuda"), out=y)
    assert bitwise_equal(host(y), np.zeros(4)) and float(s.item()) == 0.0


def test_gemv_dot_rejects_bf16_and_overlap():
    from paper_1409_0669_amd import ops
    A, _ = mat(8, 8, "bf16", 49)
    x, _ = vec(8, "bf16", 50)
    with pytest.raises(ops.BwlaError, match="UNSUPPORTED"):
        ops.gemv_dot(A, x)
    A, _ = mat(8, 8, "f64", 49)
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(ops.BwlaError, match="INVALID_ARG"):
        ops.gemv_dot(A, buf[:8], buf[:8], out=buf[4:12])  # y overlaps x and w
