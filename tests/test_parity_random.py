"""Seeded randomised parity sweep against the oracle.

Each case draws its own shape, storage type, accumulation mode, layout,
increments and library configuration from a fixed seed, so a failure names a
reproducible case.  The configurations span the whole valid space, including
ones the tuner never picks (one-lane groups, huge grids, ragged splits,
work-group counts that turn into odd splits), on shapes with ragged tails and
padded leading dimensions.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
from tests.batch_util import check as check_batch
from tests.batch_util import from_sizes
from tests.criteria import TOL, bitwise_equal, check_scalar, check_vector, cond_scale, plain_reduced
from tests.gpu_util import DT, host, mat, need_gpu, vec

pytestmark = pytest.mark.gpu

CODE = {"f64": 0, "f32": 1, "bf16": 2}
OUT = {"f64": 0, "f32": 1, "bf16": 1}
DTYPES = ("f64", "f32", "bf16")
ACCS = ("plain", "compensated")


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()
    from paper_1409_0669_amd import ops
    ops.reset_config()
    yield
    ops.reset_config()


def _rng(kind, case):
    return np.random.default_rng([2014, kind, case])


def _logint(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def _pick(rng, seq):
    return seq[int(rng.integers(len(seq)))]


def _rows_cfg(rng):
    c = dict(block=64 * int(rng.integers(1, 17)), vec=_pick(rng, (1, 2, 4, 8, 16)), rows=_pick(rng, (1, 2, 4, 8)),
             unroll=_pick(rng, (1, 2)))
    if rng.random() < 0.5:
        c["split"] = int(rng.integers(1, 10))
    else:
        c.update(split=0, grid=_pick(rng, (0, 1, 37, 256, 1000, 5000)))
    return c


def _cols_cfg(rng):
    c = dict(block=64 * int(rng.integers(1, 17)), vec=_pick(rng, (1, 2, 4, 8, 16)),
             unroll=_pick(rng, (1, 2, 4, 8)))
    if rng.random() < 0.5:
        c["split"] = int(rng.integers(1, 10))
    else:
        c.update(split=0, grid=_pick(rng, (0, 1, 37, 256, 1000, 5000)))
    return c


def _vec_cfg(rng, reduction):
    return dict(block=64 * int(rng.integers(1, 17)), vec=_pick(rng, (1, 2, 4, 8, 16)),
                unroll=_pick(rng, (1, 2, 4, 8) if reduction else (1, 2, 4)),
                grid=_pick(rng, (0, 1, 3, 256, 2049, 20000)), increment=int(rng.integers(2)))


@pytest.mark.parametrize("case", range(200))
def test_random_gemv(case):
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    rng = _rng(1, case)
    dtype, acc = _pick(rng, DTYPES), _pick(rng, ACCS)
    layout, trans = _pick(rng, ("row", "col")), int(rng.integers(2))
    m, n = _logint(rng, 1, 3000), _logint(rng, 1, 3000)
    pad = _pick(rng, (0, 0, 1, 7, 64))
    rows, cols = _rows_cfg(rng), _cols_cfg(rng)
    what = "case %d: %s %s %s trans=%d %dx%d pad=%d rows=%s cols=%s" % (case, dtype, acc, layout, trans, m, n, pad,
                                                                       rows, cols)
    ops.set_config(L.OP_GEMV_ROWS, DT[dtype], -1, **rows)
    ops.set_config(L.OP_GEMV_COLS, DT[dtype], -1, **cols)
    A, A64 = mat(m, n, dtype, 70 + case % 5, layout=layout, pad=pad)
    x, x64 = vec(m if trans else n, dtype, 75 + case % 5)
    y = ops.gemv(A, x, trans=bool(trans), acc=acc)
    B = A64.T if trans else A64
    ref = oracle.gemv(np.ascontiguousarray(B), x64)
    check_vector(host(y), ref, np.abs(B) @ np.abs(x64), TOL[dtype], what, plain_f32=plain_reduced(dtype, acc))


@pytest.mark.parametrize("case", range(200))
def test_random_reduction(case):
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    rng = _rng(2, case)
    dtype, acc = _pick(rng, DTYPES), _pick(rng, ACCS)
    op = _pick(rng, ("dot", "nrm2", "asum"))
    n = 0 if rng.random() < 0.05 else _logint(rng, 1, 3_000_000)
    incx, incy = _pick(rng, (1, 1, 1, 2, -1, -3)), _pick(rng, (1, 1, 2, -1, 0))
    cfg = _vec_cfg(rng, True)
    what = "case %d: %s %s %s n=%d incx=%d incy=%d cfg=%s" % (case, op, dtype, acc, n, incx, incy, cfg)
    ops.set_config(L.OP_DOT, DT[dtype], -1, **cfg)
    ops.set_config(L.OP_NRM2, DT[dtype], -1, **cfg)
    x, x64 = vec(1 if n == 0 else (n - 1) * abs(incx) + 1, dtype, 80 + case % 5)
    y, y64 = vec(1 if n == 0 else (n - 1) * abs(incy) + 1, dtype, 85 + case % 5)
    od = torch.float64 if dtype == "f64" else torch.float32
    out = torch.full((1,), -7.0, dtype=od, device="cuda")
    wsn = ops.workspace_size(L.OP_DOT, DT[dtype], acc, n=n)
    ws, wsb = ops._ws_ptr(ops.workspace(wsn, torch.device("cuda")))
    a = L.ACC_COMPENSATED if acc == "compensated" else L.ACC_PLAIN
    xs = oracle.strided(x64, n, incx)
    if op == "dot":
        L.check(L.lib.bwla_dot_strided(CODE[dtype], a, n, x.data_ptr(), incx, y.data_ptr(), incy, OUT[dtype],
                                       out.data_ptr(), ws, wsb, ops._stream()))
        ys = oracle.strided(y64, n, incy)
        check_scalar(float(out.item()), oracle.dot(xs, ys), cond_scale(dtype, acc, np.abs(xs * ys).sum()), TOL[dtype],
                     what)
    elif op == "nrm2":
        L.check(L.lib.bwla_nrm2_strided(CODE[dtype], a, n, x.data_ptr(), incx, OUT[dtype], out.data_ptr(), ws, wsb,
                                        ops._stream()))
        check_scalar(float(out.item()), oracle.nrm2(xs), 0.0, TOL[dtype], what)
    else:
        L.check(L.lib.bwla_asum(CODE[dtype], a, n, x.data_ptr(), incx, OUT[dtype], out.data_ptr(), ws, wsb,
                                ops._stream()))
        check_scalar(float(out.item()), oracle.asum(xs), 0.0, TOL[dtype], what)


@pytest.mark.parametrize("case", range(120))
def test_random_axpby_bitwise(case):
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    rng = _rng(3, case)
    dtype = _pick(rng, DTYPES)
    n = _logint(rng, 1, 2_000_000)
    incy, incz = _pick(rng, (1, 1, 2, -1, 0)), _pick(rng, (1, 1, -2, 3, 0))
    incx = _pick(rng, (1, 1, 2, -3))
    alpha, beta = float(rng.uniform(-2, 2)), _pick(rng, (0.0, 1.0, float(rng.uniform(-2, 2))))
    cfg = _vec_cfg(rng, False)
    what = "case %d: %s n=%d incs=%d,%d,%d a=%r b=%r cfg=%s" % (case, dtype, n, incy, incz, incx, alpha, beta, cfg)
    ops.set_config(L.OP_AXPBY, DT[dtype], -1, **cfg)
    y, y64 = vec((n - 1) * abs(incy) + 1, dtype, 90 + case % 5)
    z, z64 = vec((n - 1) * abs(incz) + 1, dtype, 95 + case % 5)
    x, x64 = vec((n - 1) * abs(incx) + 1, dtype, 100 + case % 5)
    L.check(L.lib.bwla_axpby_strided(CODE[dtype], n, alpha, None, y.data_ptr(), incy, beta, None, z.data_ptr(), incz,
                                     x.data_ptr(), incx, ops._stream()))
    vals = oracle.axpby(dtype, oracle.scalar(dtype, alpha), oracle.strided(y64, n, incy), oracle.scalar(dtype, beta),
                        oracle.strided(z64, n, incz))
    assert bitwise_equal(host(x), oracle.scatter(x64, vals, incx)), what


@pytest.mark.parametrize("case", range(40))
def test_random_batch(case):
    from paper_1409_0669_amd.batch import BatchPlan
    rng = _rng(4, case)
    dtype, acc = _pick(rng, DTYPES), _pick(rng, ACCS)
    ng, nd = int(rng.integers(1, 41)), int(rng.integers(0, 61))
    Ms = np.array([_logint(rng, 1, 1500) for _ in range(ng)])
    Ns = np.array([_logint(rng, 1, 20000 if rng.random() < 0.2 else 1500) for _ in range(ng)])
    Ds = np.array([0 if rng.random() < 0.05 else _logint(rng, 1, 200_000) for _ in range(nd)])
    align, block = _pick(rng, (1, 3, 8, 64)), _pick(rng, (64, 128, 256, 512))
    what = "case %d: %s %s %d gemvs %d dots align=%d block=%d" % (case, dtype, acc, ng, nd, align, block)
    gemvs, dots = from_sizes(dtype, Ms, Ns, Ds, seed=case, align=align)
    plan = BatchPlan(gemvs, dots, acc=acc, block=block)
    plan.run()
    torch.cuda.synchronize()
    try:
        check_batch(dtype, acc, gemvs, dots)
    except AssertionError as e:
        raise AssertionError("%s: %s" % (what, e)) from None


def _strided_buf(n, inc, dtype, stream):
    return vec(1 if n == 0 else (n - 1) * abs(inc) + 1, dtype, stream)


@pytest.mark.parametrize("case", range(100))
def test_random_gemv_ex(case):
    """y <- alpha op(A) x + beta y with increments on x and y: the GEMV of
    the oracle rounded to the output type, then its scaled addition; entries
    of y between the strided elements stay untouched."""
    import ctypes

    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    rng = _rng(5, case)
    dtype, acc = _pick(rng, DTYPES), _pick(rng, ACCS)
    layout, trans = _pick(rng, ("row", "col")), int(rng.integers(2))
    m, n = _logint(rng, 1, 2000), _logint(rng, 1, 2000)
    pad = _pick(rng, (0, 1, 5))
    incx, incy = _pick(rng, (1, 2, -1, -3)), _pick(rng, (1, 3, -1, -2))
    alpha = _pick(rng, (1.0, -1.0, 0.0, float(rng.uniform(-3, 3))))
    beta = _pick(rng, (0.0, 1.0, float(rng.uniform(-3, 3))))
    rows, cols = _rows_cfg(rng), _cols_cfg(rng)
    od = "f64" if dtype == "f64" else "f32"
    what = "case %d: %s %s %s trans=%d %dx%d pad=%d incs=%d,%d a=%r b=%r rows=%s cols=%s" % (
        case, dtype, acc, layout, trans, m, n, pad, incx, incy, alpha, beta, rows, cols)
    ops.set_config(L.OP_GEMV_ROWS, DT[dtype], -1, **rows)
    ops.set_config(L.OP_GEMV_COLS, DT[dtype], -1, **cols)
    A, A64 = mat(m, n, dtype, 70 + case % 5, layout=layout, pad=pad)
    out_len, in_len = (n, m) if trans else (m, n)
    x, x64 = _strided_buf(in_len, incx, dtype, 75 + case % 5)
    y, y64 = _strided_buf(out_len, incy, od, 80 + case % 5)
    lda = A.stride(0) if layout == "row" else A.stride(1)
    lay = L.ROW_MAJOR if layout == "row" else L.COL_MAJOR
    nbytes = ctypes.c_size_t()
    L.check(L.lib.bwla_gemv_ex_workspace_size(CODE[dtype], CODE[od], lay, trans, m, n, ctypes.byref(nbytes)))
    ws, wsn = ops._ws_ptr(ops.workspace(nbytes.value, torch.device("cuda")))
    L.check(L.lib.bwla_gemv_ex(CODE[dtype], L.ACC_COMPENSATED if acc == "compensated" else L.ACC_PLAIN, lay, trans,
                               m, n, alpha, A.data_ptr(), lda, x.data_ptr(), incx, beta, CODE[od], y.data_ptr(), incy,
                               ws, wsn, ops._stream()))
    B = np.ascontiguousarray(A64.T if trans else A64)
    xs, ys = oracle.strided(x64, in_len, incx), oracle.strided(y64, out_len, incy)
    ref = oracle.gemv_axpby(od, alpha, B, xs, beta, ys)
    scale = abs(alpha) * (np.abs(B) @ np.abs(xs)) + abs(beta) * np.abs(ys)
    got = host(y)
    check_vector(oracle.strided(got, out_len, incy), ref, scale, TOL[dtype], what, plain_f32=plain_reduced(dtype, acc))
    mask = np.ones(got.size, bool)
    mask[oracle._positions(out_len, incy)] = False
    assert bitwise_equal(got[mask], y64[mask]), what


@pytest.mark.parametrize("case", range(80))
def test_random_gemv_dot(case):
    """(y, <w, y>) in one launch sequence: y as the oracle's GEMV stored in
    A's type, the inner product within 2 tol sum_i |w_i| (|op(A)| |x|)_i of
    the oracle's <w, y>, and y bitwise what the GEMV alone stores."""
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    rng = _rng(6, case)
    dtype, acc = _pick(rng, ("f64", "f32")), _pick(rng, ACCS)
    layout, trans = _pick(rng, ("row", "col")), int(rng.integers(2))
    m, n = _logint(rng, 1, 3000), _logint(rng, 1, 3000)
    pad = _pick(rng, (0, 0, 3, 64))
    rows, cols = _rows_cfg(rng), _cols_cfg(rng)
    what = "case %d: %s %s %s trans=%d %dx%d pad=%d rows=%s cols=%s" % (case, dtype, acc, layout, trans, m, n, pad,
                                                                       rows, cols)
    ops.set_config(L.OP_GEMV_ROWS, DT[dtype], -1, **rows)
    ops.set_config(L.OP_GEMV_COLS, DT[dtype], -1, **cols)
    A, A64 = mat(m, n, dtype, 70 + case % 5, layout=layout, pad=pad)
    x, x64 = vec(m if trans else n, dtype, 75 + case % 5)
    w, w64 = vec(n if trans else m, dtype, 80 + case % 5)
    y, s = ops.gemv_dot(A, x, w, trans=bool(trans), acc=acc)
    B = np.ascontiguousarray(A64.T if trans else A64)
    ref_y, ref_s = oracle.gemv_dot(dtype, B, x64, w64)
    scale = np.abs(B) @ np.abs(x64)
    check_vector(host(y), ref_y, scale, TOL[dtype], what + " y", plain_f32=plain_reduced(dtype, acc))
    check_scalar(float(s.item()), ref_s, 2.0 * float(np.abs(w64) @ scale), TOL[dtype], what + " s")
    assert bitwise_equal(host(y), host(ops.gemv(A, x, trans=bool(trans), acc=acc))), what


@pytest.mark.parametrize("case", range(60))
def test_random_ger_bitwise(case):
    """A <- u v^T: every entry rounded once, padding between lines untouched."""
    from paper_1409_0669_amd import ops
    rng = _rng(7, case)
    dtype, layout = _pick(rng, DTYPES), _pick(rng, ("row", "col"))
    m, n = _logint(rng, 1, 3000), _logint(rng, 1, 3000)
    pad = _pick(rng, (0, 1, 7, 64))
    what = "case %d: %s %s %dx%d pad=%d" % (case, dtype, layout, m, n, pad)
    A, _ = mat(m, n, dtype, 70 + case % 5, layout=layout, pad=pad)
    u, u64 = vec(m, dtype, 75 + case % 5)
    v, v64 = vec(n, dtype, 80 + case % 5)
    base = A.t() if layout == "col" else A
    before = host(base.as_strided((base.shape[0], base.stride(0)), (base.stride(0), 1)).contiguous())
    ops.ger(u, v, A)
    after = host(base.as_strided((base.shape[0], base.stride(0)), (base.stride(0), 1)).contiguous())
    lda = base.stride(0)
    ref = oracle.ger(dtype, u64, v64, layout=0 if layout == "row" else 1, lda=lda).reshape(-1, lda)
    lines = base.shape[1]
    assert bitwise_equal(after[:, :lines], ref[:, :lines]), what
    assert bitwise_equal(after[:, lines:], before[:, lines:]), what


@pytest.mark.parametrize("case", range(60))
def test_random_cg_update(case):
    """x <- x + a p, r <- r - a q bitwise the oracle's scaled additions, and
    <r, r> of the new r within tolerance, under random configurations."""
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    rng = _rng(8, case)
    dtype, acc = _pick(rng, DTYPES), _pick(rng, ACCS)
    n = _logint(rng, 1, 2_000_000)
    alpha = float(rng.uniform(-2, 2))
    cfg = _vec_cfg(rng, True)
    what = "case %d: %s %s n=%d a=%r cfg=%s" % (case, dtype, acc, n, alpha, cfg)
    ops.set_config(L.OP_CG, DT[dtype], -1, **cfg)
    x, x64 = vec(n, dtype, 70 + case % 5, dist="normal")
    p, p64 = vec(n, dtype, 75 + case % 5, dist="normal")
    r, r64 = vec(n, dtype, 80 + case % 5, dist="normal")
    q, q64 = vec(n, dtype, 85 + case % 5, dist="normal")
    rr = float(ops.cg_update(alpha, x, p, r, q, acc=acc).item())
    ae = oracle.scalar(dtype, alpha)
    rref = oracle.axpby(dtype, -ae, q64, 1.0, r64)
    assert bitwise_equal(host(x), oracle.axpby(dtype, ae, p64, 1.0, x64)), what
    assert bitwise_equal(host(r), rref), what
    check_scalar(rr, oracle.dot(rref, rref), 0.0, TOL[dtype], what)


@pytest.mark.parametrize("case", range(100))
def test_random_misaligned_unit_stride(case):
    """Unit-stride vectors that start anywhere in their allocations (0 to 7
    elements past a 256-byte boundary, independently per operand) under
    random configurations: the pack width then falls back per call.  copy,
    axpby and scal_to bitwise, dot and nrm2 within the criteria, and the
    guard entries around the output untouched."""
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    rng = _rng(10, case)
    dtype, acc = _pick(rng, DTYPES), _pick(rng, ACCS)
    n = _logint(rng, 1, 1_000_000)
    oy, oz, ox = (int(rng.integers(0, 8)) for _ in range(3))
    ecfg, rcfg = _vec_cfg(rng, False), _vec_cfg(rng, True)
    a, b = float(rng.uniform(-2, 2)), float(rng.uniform(-2, 2))
    what = "case %d: %s %s n=%d offsets y=%d z=%d x=%d elem=%s red=%s" % (case, dtype, acc, n, oy, oz, ox, ecfg, rcfg)
    for op in (L.OP_AXPBY, L.OP_COPY):
        ops.set_config(op, DT[dtype], -1, **ecfg)
    for op in (L.OP_DOT, L.OP_NRM2):
        ops.set_config(op, DT[dtype], -1, **rcfg)
    y, y64 = vec(n, dtype, 110 + case % 5, pad_front=oy)
    z, z64 = vec(n, dtype, 115 + case % 5, pad_front=oz)
    buf = torch.full((n + ox + 8,), float("nan"), dtype=DT[dtype], device="cuda")
    x = buf[ox:ox + n]
    ops.axpby(a, y, b, z, out=x)
    ref = oracle.axpby(dtype, oracle.scalar(dtype, a), y64, oracle.scalar(dtype, b), z64)
    assert bitwise_equal(host(x), ref), what
    ops.copy(z, out=x)
    assert bitwise_equal(host(x), z64), what
    ops.scal_to(a, y, out=x)
    assert bitwise_equal(host(x), oracle.scal(dtype, oracle.scalar(dtype, a), y64)), what
    rest = torch.cat([buf[:ox], buf[ox + n:]])
    assert bool(torch.isnan(rest).all()), what
    check_scalar(float(ops.dot(y, z, acc=acc).item()), oracle.dot(y64, z64),
                 cond_scale(dtype, acc, np.abs(y64 * z64).sum()), TOL[dtype], "dot " + what)
    check_scalar(float(ops.nrm2(y, acc=acc).item()), oracle.nrm2(y64), 0.0, TOL[dtype], "nrm2 " + what)
