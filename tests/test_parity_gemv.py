"""GPU parity of the matrix-vector products (both layouts, both transposes)
and of the rank-1 overwrite, against the oracle."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from tests.criteria import TOL, bitwise_equal, check_vector, plain_reduced
from tests.gpu_util import DT, guarded, host, mat, need_gpu, vec

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 7), (7, 1), (33, 65), (128, 256), (257, 1023), (1000, 3001), (64, 20000), (5000, 40)]
DTYPES = ["f64", "f32", "bf16"]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()
    from paper_1409_0669_amd import ops
    ops.reset_config()
    yield
    ops.reset_config()


def _ref(A64, x64, trans):
    B = A64.T if trans else A64
    y = oracle.gemv(np.ascontiguousarray(B), x64)
    scale = np.abs(B) @ np.abs(x64)
    return y, scale


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("layout", ["row", "col"])
@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_gemv(dtype, layout, trans, shape):
    from paper_1409_0669_amd import ops
    m, n = shape
    A, A64 = mat(m, n, dtype, 21, layout=layout)
    x, x64 = vec(m if trans else n, dtype, 22)
    for acc in ("plain", "compensated"):
        y, guard = guarded(n if trans else m, ops.default_out_dtype(DT[dtype]))
        ops.gemv(A, x, trans=bool(trans), acc=acc, out=y)
        ref, scale = _ref(A64, x64, trans)
        what = "%s %s t=%d %s" % (dtype, layout, trans, acc)
        check_vector(host(y), ref, scale, TOL[dtype], what, plain_f32=plain_reduced(dtype, acc))
        guard(what)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["row", "col"])
@pytest.mark.parametrize("trans", [0, 1])
def test_gemv_padded_lda_and_f64_output(dtype, layout, trans):
    from paper_1409_0669_amd import ops
    m, n = 301, 517
    A, A64 = mat(m, n, dtype, 23, layout=layout, pad=5)
    x, x64 = vec(m if trans else n, dtype, 24)
    y = ops.gemv(A, x, trans=bool(trans), out_dtype=torch.float64)
    assert y.dtype == torch.float64
    ref, scale = _ref(A64, x64, trans)
    check_vector(host(y), ref, scale, TOL[dtype])


@pytest.mark.parametrize("layout", ["row", "col"])
def test_gemv_identity_permutation_rank_one(layout):
    from paper_1409_0669_amd import ops
    n = 777
    I = torch.eye(n, dtype=torch.float64, device="cuda")
    if layout == "col":
        I = I.t().contiguous().t()
    x, x64 = vec(n, "f64", 25)
    assert bitwise_equal(host(ops.gemv(I, x)), x64)
    perm = np.random.default_rng(4).permutation(n)
    P = torch.from_numpy(np.eye(n)[perm]).cuda()
    if layout == "col":
        P = P.t().contiguous().t()
    assert bitwise_equal(host(ops.gemv(P, x)), x64[perm])
    assert bitwise_equal(host(ops.gemv(P, x, trans=True)), x64[np.argsort(perm)])
    rng = np.random.default_rng(5)
    u = rng.integers(-9, 10, 300).astype(np.float64)
    v = rng.integers(-9, 10, 200).astype(np.float64)
    xi = rng.integers(-9, 10, 200).astype(np.float64)
    R = torch.from_numpy(np.outer(u, v)).cuda()
    if layout == "col":
        R = R.t().contiguous().t()
    assert bitwise_equal(host(ops.gemv(R, torch.from_numpy(xi).cuda())), u * float(v @ xi))


def test_gemv_empty():
    from paper_1409_0669_amd import ops
    A = torch.zeros(4, 0, dtype=torch.float64, device="cuda")
    y = ops.gemv(A, torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert bitwise_equal(host(y), np.zeros(4))
    A = torch.zeros(0, 6, dtype=torch.float32, device="cuda")
    assert ops.gemv(A, torch.zeros(6, dtype=torch.float32, device="cuda")).numel() == 0


# the last two of each list give a work-group count instead of a split: the
# split then follows each shape (ceil(grid / output tiles)), ragged counts
ROWS_CFG = [dict(block=64, vec=1, rows=1, split=1), dict(block=128, vec=2, rows=2, split=3, unroll=2),
            dict(block=256, vec=4, rows=8, split=1, unroll=2), dict(block=1024, vec=16, rows=4, split=2),
            dict(block=512, vec=8, rows=1, split=7, unroll=2),
            dict(block=256, vec=4, rows=4, split=0, grid=1000, unroll=2), dict(block=128, vec=2, rows=8, grid=37),
            dict(block=512, vec=4, rows=2, split=0, unroll=2), dict(block=256, vec=1, rows=4, split=5)]
COLS_CFG = [dict(block=64, vec=1, unroll=1, split=1), dict(block=128, vec=2, unroll=2, split=3),
            dict(block=256, vec=4, unroll=4, split=1), dict(block=1024, vec=16, unroll=4, split=2),
            dict(block=512, vec=8, unroll=1, split=9),
            dict(block=256, vec=2, unroll=8, split=0, grid=700), dict(block=512, vec=4, unroll=2, grid=33),
            # 32 and 16 lines in flight (halved where they would hold more
            # than 128 bytes of A per lane)
            dict(block=1024, vec=1, unroll=32, split=0, grid=256), dict(block=512, vec=2, unroll=16, split=3)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("cfg", range(len(ROWS_CFG)))
def test_gemv_configs(dtype, cfg):
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    ops.set_config(L.OP_GEMV_ROWS, DT[dtype], -1, **ROWS_CFG[cfg])
    ops.set_config(L.OP_GEMV_COLS, DT[dtype], -1, **COLS_CFG[cfg])
    for (m, n) in [(37, 3000), (2500, 131), (513, 515)]:
        for layout in ("row", "col"):
            A, A64 = mat(m, n, dtype, 26, layout=layout)
            for trans in (0, 1):
                x, x64 = vec(m if trans else n, dtype, 27)
                for acc in ("plain", "compensated"):
                    y, guard = guarded(n if trans else m, ops.default_out_dtype(DT[dtype]))
                    ops.gemv(A, x, trans=bool(trans), acc=acc, out=y)
                    ref, scale = _ref(A64, x64, trans)
                    what = "%s %s %s %s" % (cfg, layout, trans, acc)
                    check_vector(host(y), ref, scale, TOL[dtype], what, plain_f32=plain_reduced(dtype, acc))
                    guard(what)


@pytest.mark.parametrize("acc", ["plain", "compensated"])
@pytest.mark.parametrize("shape", [(4096, 4096), (16384, 2048), (2048, 16384)])
def test_gemv_shipped_table_on_differentiation_shapes(acc, shape):
    """The shipped table's GEMV entries (work-group counts that the split
    follows on each shape) on the f32 shapes of the differentiation workload:
    y = A x and dx = A^T ybar against the oracle, every output."""
    from paper_1409_0669_amd import ops
    assert ops.load_default_tuning()
    m, n = shape
    A, A64 = mat(m, n, "f32", 28, layout="row")
    for trans in (0, 1):
        x, x64 = vec(m if trans else n, "f32", 29)
        y = ops.gemv(A, x, trans=bool(trans), acc=acc)
        ref, scale = _ref(A64, x64, trans)
        check_vector(host(y), ref, scale, TOL["f32"], "%s %s trans=%d" % (acc, shape, trans),
                     plain_f32=plain_reduced("f32", acc))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("acc", ["plain", "compensated"])
def test_gemv_rows_unroll_keeps_the_order(dtype, acc):
    """Two packs per line in flight take each line's packs in the same order
    as one: the results are bitwise the same (with and without a split)."""
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    A, _ = mat(1500, 9001, dtype, 39)
    x, _ = vec(9001, dtype, 40)
    for split in (1, 3):
        got = []
        for u in (1, 2):
            ops.set_config(L.OP_GEMV_ROWS, DT[dtype], -1, block=256, rows=2, unroll=u, split=split)
            got.append(host(ops.gemv(A, x, acc=acc)))
        assert bitwise_equal(got[0], got[1]), split


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("acc", ["plain", "compensated"])
def test_gemv_cols_wave_combine_paths_agree(dtype, acc):
    """The cols kernel adds its waves' partials in wave order whether they
    meet in dynamic LDS after one barrier (512 threads, 2-wide packs: 14 KiB)
    or pass one wave at a time (8-wide packs: 56 KiB, over the 32 KiB limit);
    pack width and unroll do not change which wave takes which line.  All
    results are bitwise the same, with and without a split."""
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    m, n = 3000, 2500  # lda = 3000 keeps 8-wide packs aligned
    A, _ = mat(m, n, dtype, 41, layout="col")
    x, _ = vec(n, dtype, 42)
    for split in (1, 3):
        got = []
        for v, u in ((2, 4), (8, 4), (8, 1)):
            ops.set_config(L.OP_GEMV_COLS, DT[dtype], -1, block=512, vec=v, unroll=u, split=split)
            assert ops.get_config(L.OP_GEMV_COLS, DT[dtype], m, n, acc=acc)["vec"] == v
            got.append(host(ops.gemv(A, x, acc=acc)))
        assert bitwise_equal(got[0], got[1]) and bitwise_equal(got[0], got[2]), split


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gemv_deterministic(dtype):
    from paper_1409_0669_amd import ops
    for layout in ("row", "col"):
        A, _ = mat(3000, 2000, dtype, 28, layout=layout)
        x, _ = vec(2000, dtype, 29)
        first = host(ops.gemv(A, x))
        for _ in range(5):
            assert bitwise_equal(host(ops.gemv(A, x)), first)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("layout", ["row", "col"])
@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (64, 64), (129, 1031), (2000, 77)])
def test_ger_bitwise(dtype, layout, shape):
    from paper_1409_0669_amd import ops
    m, n = shape
    u, u64 = vec(m, dtype, 31)
    v, v64 = vec(n, dtype, 32)
    A, _ = mat(m, n, dtype, 33, layout=layout, pad=3)
    ops.ger(u, v, A)
    got = host(A.t() if layout == "col" else A)
    ref = oracle.ger(dtype, u64, v64, layout=oracle.ROW_MAJOR if layout == "row" else oracle.COL_MAJOR)
    ref = ref.reshape(m, n) if layout == "row" else ref.reshape(n, m)
    assert bitwise_equal(got, ref)


@pytest.mark.parametrize("dtype", DTYPES)
def test_ger_padding_untouched(dtype):
    from paper_1409_0669_amd import ops
    m, n, pad = 50, 70, 6
    buf = torch.full((m, n + pad), 7.0, dtype=DT[dtype], device="cuda")
    u, u64 = vec(m, dtype, 34)
    v, v64 = vec(n, dtype, 35)
    ops.ger(u, v, buf[:, :n])
    assert torch.all(buf[:, n:] == 7.0)


GER_CFG = [dict(block=64, vec=1, rows=1), dict(block=128, vec=2, rows=8), dict(block=1024, vec=16, rows=4),
           dict(block=512, vec=4, rows=2)]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("cfg", range(len(GER_CFG)))
def test_ger_configs_bitwise(dtype, cfg):
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    ops.set_config(L.OP_GER, DT[dtype], -1, **GER_CFG[cfg])
    for (m, n) in [(37, 3001), (1029, 65)]:
        for layout in ("row", "col"):
            u, u64 = vec(m, dtype, 36)
            v, v64 = vec(n, dtype, 37)
            A, _ = mat(m, n, dtype, 38, layout=layout, pad=2)
            ops.ger(u, v, A)
            got = host(A.t() if layout == "col" else A)
            ref = oracle.ger(dtype, u64, v64, layout=oracle.ROW_MAJOR if layout == "row" else oracle.COL_MAJOR)
            ref = ref.reshape(m, n) if layout == "row" else ref.reshape(n, m)
            assert bitwise_equal(got, ref), (cfg, m, n, layout)
