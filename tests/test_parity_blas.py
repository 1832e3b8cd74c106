"""GPU parity of the BLAS-style additions against the oracle: vectors with
increments (positive, negative, zero for inputs), scal, asum, GEMV with
alpha/beta and strided x/y, and sums with infinite or NaN entries.

Negative increments cannot be expressed as torch views, so these tests call
the C ABI with raw device pointers; the torch-level entry points are checked
on strided views at the end."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle
from tests.criteria import TOL, bitwise_equal, check_scalar, check_vector, cond_scale, plain_reduced
from tests.gpu_util import DT, guarded, host, mat, need_gpu, vec

pytestmark = pytest.mark.gpu

CODE = {"f64": 0, "f32": 1, "bf16": 2}
OUT = {"f64": 0, "f32": 1, "bf16": 1}  # default reduction output type
INCS = [(2, 1), (1, 3), (-1, 1), (3, -2), (0, 1), (-2, -2), (5, 7)]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()
    from paper_1409_0669_amd import ops
    ops.reset_config()
    yield
    ops.reset_config()


def _lib():
    from paper_1409_0669_amd import _lib as L
    return L


def _stream():
    from paper_1409_0669_amd import ops
    return ops._stream()


def _check(status):
    _lib().check(status)


def _buf(n, inc, dtype, stream):
    """A device buffer holding a strided vector of n elements: (tensor, f64 values)."""
    length = 1 if n == 0 else (n - 1) * abs(inc) + 1
    return vec(length, dtype, stream)


def _out_buf(n, inc, dtype, stream):
    """As _buf, for an output: the buffer sits between sentinel slack;
    returns (tensor, f64 values, guard check)."""
    t, t64 = _buf(n, inc, dtype, stream)
    out, guard = guarded(t.numel(), dtype)
    out.copy_(t)
    return out, t64, guard


def _ws(nbytes):
    from paper_1409_0669_amd import ops
    return ops._ws_ptr(ops.workspace(nbytes, torch.device("cuda")))


def _red_ws(dtype, n):
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    return _ws(ops.workspace_size(L.OP_DOT, DT[dtype], n=n))


# ---------------------------------------------------------------------------
# elementwise: bitwise
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [1, 7, 1000, 100003])
@pytest.mark.parametrize("incs", INCS)
def test_copy_strided_bitwise(dtype, n, incs):
    incy, incx = incs
    y, y64 = _buf(n, incy, dtype, 61)
    x, x64, guard = _out_buf(n, incx, dtype, 62)
    _check(_lib().lib.bwla_copy_strided(CODE[dtype], n, y.data_ptr(), incy, x.data_ptr(), incx, _stream()))
    ref = oracle.scatter(x64, oracle.copy(oracle.strided(y64, n, incy)), incx)
    assert bitwise_equal(host(x), ref)  # every entry, the gaps included
    guard("copy_strided")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [1, 1000, 65537])
@pytest.mark.parametrize("incs", [(2, 3, 1), (-1, 1, -1), (1, 0, 2), (3, -3, -2), (4, 4, 4)])
def test_axpby_strided_bitwise(dtype, n, incs):
    incy, incz, incx = incs
    y, y64 = _buf(n, incy, dtype, 63)
    z, z64 = _buf(n, incz, dtype, 64)
    x, x64, guard = _out_buf(n, incx, dtype, 65)
    a, b = 0.75, -1.3
    _check(_lib().lib.bwla_axpby_strided(CODE[dtype], n, a, None, y.data_ptr(), incy, b, None, z.data_ptr(), incz,
                                         x.data_ptr(), incx, _stream()))
    vals = oracle.axpby(dtype, oracle.scalar(dtype, a), oracle.strided(y64, n, incy), oracle.scalar(dtype, b),
                        oracle.strided(z64, n, incz))
    assert bitwise_equal(host(x), oracle.scatter(x64, vals, incx))
    guard("axpby_strided")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_axpby_strided_in_place_and_device_scalars(dtype):
    """r -= a q on every third element, a on the device; the output aliases z
    exactly (same pointer and increment)."""
    n, inc = 5001, 3
    r, r64 = _buf(n, inc, dtype, 66)
    q, q64 = _buf(n, -2, dtype, 67)
    cd = torch.float64 if dtype == "f64" else torch.float32
    adev = torch.tensor([0.5], dtype=cd, device="cuda")
    _check(_lib().lib.bwla_axpby_strided(CODE[dtype], n, -3.0, adev.data_ptr(), q.data_ptr(), -2, 1.0, None,
                                         r.data_ptr(), inc, r.data_ptr(), inc, _stream()))
    a = oracle.scalar(dtype, -3.0, 0.5)
    vals = oracle.axpby(dtype, a, oracle.strided(q64, n, -2), 1.0, oracle.strided(r64, n, inc))
    assert bitwise_equal(host(r), oracle.scatter(r64, vals, inc))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [1, 9, 4099, 1 << 20])
@pytest.mark.parametrize("inc", [1, 2, -3])
def test_scal_bitwise(dtype, n, inc):
    x, x64, guard = _out_buf(n, inc, dtype, 68)
    _check(_lib().lib.bwla_scal(CODE[dtype], n, -2.5, None, x.data_ptr(), inc, _stream()))
    vals = oracle.scal(dtype, oracle.scalar(dtype, -2.5), oracle.strided(x64, n, inc))
    assert bitwise_equal(host(x), oracle.scatter(x64, vals, inc))
    guard("scal")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_scal_ieee_specials(dtype):
    from paper_1409_0669_amd import ops
    vals = [np.inf, -np.inf, np.nan, -0.0, 0.0, 3.0, -1e-30]
    x = torch.tensor(vals, dtype=DT[dtype], device="cuda")
    ops.scal(2.0, x)
    ref = oracle.scal(dtype, 2.0, np.array(vals, dtype=np.float64).astype(np.float32 if dtype == "f32" else np.float64))
    got = host(x)
    assert bitwise_equal(got, ref)
    assert np.signbit(got[3]) and not np.signbit(got[4])


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [1, 7, 4099, (1 << 20) + 3])
def test_scal_to_bitwise(dtype, n):
    """x <- a y out of place, a from the host and from a device scalar (the
    inner product's gradient form), against the oracle's one rounding per
    element; y untouched."""
    from paper_1409_0669_amd import ops
    y, y64 = vec(n, dtype, 83)
    x, guard = guarded(n, dtype)
    ops.scal_to(-2.5, y, out=x)
    assert bitwise_equal(host(x), oracle.scal(dtype, oracle.scalar(dtype, -2.5), y64))
    zb = torch.tensor([0.37], dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")
    ops.scal_to(1.0, y, out=x, alpha_dev=zb)
    assert bitwise_equal(host(x), oracle.scal(dtype, oracle.scalar(dtype, 1.0, float(zb.item())), y64))
    assert bitwise_equal(host(y), y64)
    guard("scal_to")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_scal_to_ieee_specials_and_signed_zeros(dtype):
    """One IEEE product per element: zbar * inf is an infinity, NaN stays
    NaN, -zbar * +0 = -0, and 0 * inf = NaN -- where a scaled addition with
    beta = 0 (an extra 0 * y term) gives NaN and +0."""
    from paper_1409_0669_amd import ops
    vals = np.array([np.inf, -np.inf, np.nan, -0.0, 0.0, 3.0, -0.5])
    y = torch.tensor(vals, dtype=DT[dtype], device="cuda")
    for a in (-2.0, 0.5, 0.0, -0.0):
        zb = torch.tensor([a], dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")
        x = ops.scal_to(1.0, y, alpha_dev=zb)
        assert bitwise_equal(host(x), oracle.scal(dtype, oracle.scalar(dtype, 1.0, a), host(y))), a


# ---------------------------------------------------------------------------
# reductions
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [1, 33, 10007, 1 << 20])
@pytest.mark.parametrize("incs", [(2, 1), (-1, 3), (1, 0), (-4, -4)])
def test_dot_strided(dtype, n, incs):
    incx, incy = incs
    x, x64 = _buf(n, incx, dtype, 69)
    y, y64 = _buf(n, incy, dtype, 70)
    xs, ys = oracle.strided(x64, n, incx), oracle.strided(y64, n, incy)
    ref, absum = oracle.dot(xs, ys), float(np.abs(xs * ys).sum())
    ws, wsn = _red_ws(dtype, n)
    for acc in (0, 1):
        out = torch.zeros((), dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")
        _check(_lib().lib.bwla_dot_strided(CODE[dtype], acc, n, x.data_ptr(), incx, y.data_ptr(), incy, OUT[dtype],
                                           out.data_ptr(), ws, wsn, _stream()))
        check_scalar(float(out.item()), ref, cond_scale(dtype, acc, absum), TOL[dtype],
                     "dot %s n=%d incs=%s acc=%d" % (dtype, n, incs, acc))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [1, 33, 10007, 1 << 20, (1 << 22) + 5])
@pytest.mark.parametrize("inc", [1, 2, -1, -3])
def test_nrm2_and_asum_strided(dtype, n, inc):
    x, x64 = _buf(n, inc, dtype, 71)
    xs = oracle.strided(x64, n, inc)
    ws, wsn = _red_ws(dtype, n)
    lib = _lib().lib
    for acc in (0, 1):
        out = torch.zeros((), dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")
        _check(lib.bwla_nrm2_strided(CODE[dtype], acc, n, x.data_ptr(), inc, OUT[dtype], out.data_ptr(), ws, wsn,
                                     _stream()))
        check_scalar(float(out.item()), oracle.nrm2(xs), 0.0, TOL[dtype], "nrm2 acc=%d" % acc)
        _check(lib.bwla_asum(CODE[dtype], acc, n, x.data_ptr(), inc, OUT[dtype], out.data_ptr(), ws, wsn, _stream()))
        check_scalar(float(out.item()), oracle.asum(xs), 0.0, TOL[dtype], "asum acc=%d" % acc)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_asum_f64_output_and_configs(dtype):
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    n = 300001
    x, x64 = vec(n, dtype, 72)
    ref = oracle.asum(x64)
    for cfg in (dict(block=64, vec=1, unroll=1, grid=1), dict(block=256, vec=2, unroll=4, grid=0),
                dict(block=1024, vec=8, unroll=2, grid=512, increment=1)):
        ops.set_config(L.OP_NRM2, DT[dtype], -1, **cfg)
        for acc in ("plain", "compensated"):
            got = ops.asum(x, acc=acc, out_dtype=torch.float64)
            check_scalar(float(got.item()), ref, 0.0, TOL[dtype], "asum %s %s" % (cfg, acc))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("acc", ["plain", "compensated"])
def test_sums_with_infinite_and_nan_entries(dtype, acc):
    """A sum with an infinite term is that infinity (NaN for inf - inf or a
    NaN term), in both accumulation modes; the compensation must not turn it
    into NaN."""
    from paper_1409_0669_amd import ops
    n = 100000
    base, b64 = vec(n, dtype, 73)
    ones = torch.ones(n, dtype=DT[dtype], device="cuda")
    cases = {"inf": [(17, np.inf)], "-inf": [(99999, -np.inf)], "inf-inf": [(5, np.inf), (70000, -np.inf)],
             "nan": [(4242, np.nan)]}
    for name, entries in cases.items():
        x, x64 = base.clone(), b64.copy()
        for i, v in entries:
            x[i] = v
            x64[i] = v
        check_scalar(float(ops.dot(x, ones, acc=acc).item()), oracle.dot(x64, np.ones(n)), 0.0, TOL[dtype],
                     "dot " + name)
        check_scalar(float(ops.asum(x, acc=acc).item()), oracle.asum(x64), 0.0, TOL[dtype], "asum " + name)
        check_scalar(float(ops.nrm2(x, acc=acc).item()), oracle.nrm2(x64), 0.0, TOL[dtype], "nrm2 " + name)
        A = x[: 300 * 300].view(300, 300)
        A64 = x64[: 300 * 300].reshape(300, 300)
        y = host(ops.gemv(A, ones[:300], acc=acc))
        ref = oracle.gemv(A64, np.ones(300))
        fin = np.isfinite(ref)
        assert bitwise_equal(y[~fin], ref[~fin]), name
        # the transposed product reads the same bytes with the cols kernel
        # (the special entry's column is non-finite)
        yt = host(ops.gemv(A, ones[:300], trans=True, acc=acc))
        reft = oracle.gemv(np.ascontiguousarray(A64.T), np.ones(300))
        fin = np.isfinite(reft)
        assert bitwise_equal(yt[~fin], reft[~fin]), name + " transposed"
        check_vector(yt[fin], reft[fin], np.abs(A64.T[fin]) @ np.ones(300), TOL[dtype], name + " transposed",
                     plain_f32=plain_reduced(dtype, acc))


# ---------------------------------------------------------------------------
# GEMV with alpha, beta and increments
# ---------------------------------------------------------------------------

GEMV_CASES = [(2.0, 0.0, 1, 1), (1.0, 0.0, 2, 1), (1.0, 0.0, 1, 3), (-0.5, 1.5, 1, 1), (1.0, -1.0, -1, 2),
              (0.25, 2.0, 3, -2), (3.0, 0.0, -2, -1)]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("layout", ["row", "col"])
@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("case", range(len(GEMV_CASES)))
def test_gemv_ex(dtype, layout, trans, case):
    from paper_1409_0669_amd import _lib as L
    alpha, beta, incx, incy = GEMV_CASES[case]
    m, n = 301, 517
    A, A64 = mat(m, n, dtype, 74, layout=layout, pad=3)
    out_len, in_len = (n, m) if trans else (m, n)
    x, x64 = _buf(in_len, incx, dtype, 75)
    od = "f64" if dtype == "f64" else "f32"
    y, y64 = _buf(out_len, incy, od, 76)
    lda = A.stride(0) if layout == "row" else A.stride(1)
    lay = L.ROW_MAJOR if layout == "row" else L.COL_MAJOR
    nbytes = ctypes.c_size_t()
    _check(L.lib.bwla_gemv_ex_workspace_size(CODE[dtype], CODE[od], lay, trans, m, n, ctypes.byref(nbytes)))
    ws, wsn = _ws(nbytes.value)
    for acc in (0, 1):
        yy, guard = guarded(y.numel(), od)
        yy.copy_(y)
        _check(L.lib.bwla_gemv_ex(CODE[dtype], acc, lay, trans, m, n, alpha, A.data_ptr(), lda, x.data_ptr(), incx,
                                  beta, CODE[od], yy.data_ptr(), incy, ws, wsn, _stream()))
        B = A64.T if trans else A64
        xs, ys = oracle.strided(x64, in_len, incx), oracle.strided(y64, out_len, incy)
        ref = oracle.gemv_axpby(od, alpha, np.ascontiguousarray(B), xs, beta, ys)
        # the stored GEMV result is within tol (|op(A)| |x|)_i of the oracle's;
        # alpha carries that, beta y is exact input
        scale = abs(alpha) * (np.abs(B) @ np.abs(xs)) + abs(beta) * np.abs(ys)
        got = host(yy)
        check_vector(oracle.strided(got, out_len, incy), ref, scale, TOL[dtype], "gemv_ex case %d acc %d" % (case, acc),
                     plain_f32=plain_reduced(dtype, acc))
        # entries between the strided elements of y are untouched
        mask = np.ones(got.size, bool)
        mask[oracle._positions(out_len, incy)] = False
        assert bitwise_equal(got[mask], y64[mask])
        guard("gemv_ex case %d acc %d" % (case, acc))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gemv_ex_is_the_composite(dtype):
    """alpha op(A) x + beta y is bitwise the library's GEMV followed by its
    axpby (beta != 0) or scal (beta == 0); with beta == 0 a NaN-filled y is
    not read."""
    from paper_1409_0669_amd import ops
    m, n = 777, 1234
    A, _ = mat(m, n, dtype, 77)
    x, _ = vec(n, dtype, 78)
    y0, _ = vec(m, dtype, 79)
    s = ops.gemv(A, x, acc="compensated")
    y = y0.clone()
    ops.gemv(A, x, acc="compensated", out=y, alpha=0.3, beta=-1.7)
    assert bitwise_equal(host(y), host(ops.axpby(0.3, s, -1.7, y0)))
    y = torch.full((m,), float("nan"), dtype=DT[dtype], device="cuda")
    ops.gemv(A, x, acc="compensated", out=y, alpha=-4.0)
    ref = s.clone()
    ops.scal(-4.0, ref)
    assert bitwise_equal(host(y), host(ref))


def test_gemv_ex_empty_reduction():
    """A zero-length reduction: op(A) x = 0, so y = alpha 0 + beta y."""
    from paper_1409_0669_amd import ops
    A = torch.zeros(5, 0, dtype=torch.float64, device="cuda")
    y = torch.arange(5, dtype=torch.float64, device="cuda")
    ops.gemv(A, torch.zeros(0, dtype=torch.float64, device="cuda"), out=y, alpha=2.0, beta=3.0)
    assert bitwise_equal(host(y), 3.0 * np.arange(5))


# ---------------------------------------------------------------------------
# torch-level strided views
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_ops_accept_strided_views(dtype):
    from paper_1409_0669_amd import ops
    n = 20001
    xb, xb64 = vec(3 * n, dtype, 80)
    yb, yb64 = vec(2 * n, dtype, 81)
    x, x64 = xb[::3], xb64[::3]
    y, y64 = yb[::2], yb64[::2]
    check_scalar(float(ops.dot(x, y).item()), oracle.dot(x64, y64), cond_scale(dtype, "plain", np.abs(x64 * y64).sum()),
                 TOL[dtype])
    check_scalar(float(ops.nrm2(x).item()), oracle.nrm2(x64), 0.0, TOL[dtype])
    check_scalar(float(ops.asum(y, acc="compensated").item()), oracle.asum(y64), 0.0, TOL[dtype])
    out = torch.zeros(2 * n, dtype=DT[dtype], device="cuda")
    ops.axpby(2.0, x, -1.0, y, out=out[1::2])
    ref = oracle.axpby(dtype, oracle.scalar(dtype, 2.0), x64, oracle.scalar(dtype, -1.0), y64)
    got = host(out)
    assert bitwise_equal(got[1::2], ref) and not got[0::2].any()
    c = ops.copy(x)
    assert c.is_contiguous() and bitwise_equal(host(c), x64)
    if dtype != "bf16":
        A, A64 = mat(n, 7, dtype, 82)
        z = torch.zeros(14, dtype=DT[dtype], device="cuda")
        ops.gemv(A, x, trans=True, out=z[::2], alpha=1.0)
        gz = host(z)
        check_vector(gz[::2], oracle.gemv(np.ascontiguousarray(A64.T), x64), np.abs(A64.T) @ np.abs(x64), TOL[dtype],
                     plain_f32=plain_reduced(dtype, "plain"))
        assert not gz[1::2].any()
