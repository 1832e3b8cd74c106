"""Parity at the full paper-scale sizes, in the launch configuration the
benchmark times (the shipped tuning table): vectors of 2^26 and 10^7 entries,
GEMV 4096^2 and 16384^2 (every output of both layouts and both transposes),
GEMV beyond 2^31 elements (sampled outputs), composites at n = 2^24 and
8192^2 with normal inputs, and the reduced-precision forms."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.criteria import TOL, bitwise_equal, check_scalar, check_vector, plain_reduced
from tests.gpu_util import host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _tuned():
    need_gpu()
    from paper_1409_0669_amd import ops
    ops.reset_config()
    assert ops.load_default_tuning()
    yield
    ops.reset_config()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [10 ** 7, 1 << 26])
def test_vectors_full(dtype, n):
    from paper_1409_0669_amd import ops
    y = W.device_draw(n, dtype, 0, 100)
    z = W.device_draw(n, dtype, 0, 200)
    x = ops.axpby(0.75, y, -1.25, z)
    y64, z64 = host(y), host(z)
    ref = oracle.axpby(dtype, oracle.scalar(dtype, 0.75), y64, oracle.scalar(dtype, -1.25), z64)
    assert bitwise_equal(host(x), ref)
    del x, ref
    for acc in ("plain", "compensated"):
        check_scalar(float(ops.dot(y, z, acc=acc).item()), oracle.dot(y64, z64), 0.0, TOL[dtype], "dot " + acc)
        check_scalar(float(ops.nrm2(y, acc=acc).item()), oracle.nrm2(y64), 0.0, TOL[dtype], "nrm2 " + acc)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("layout", ["row", "col"])
def test_gemv_4096_every_output(dtype, layout):
    from paper_1409_0669_amd import ops
    m = n = 4096
    A = W.device_draw(m * n, dtype, 0, 300).view(m, n)
    if layout == "col":
        A = A.t().contiguous().t()
    x = W.device_draw(n, dtype, 0, 400)
    A64, x64 = host(A), host(x)
    for trans in (False, True):
        y = ops.gemv(A, x, trans=trans)
        B = A64.T if trans else A64
        check_vector(host(y), oracle.gemv(np.ascontiguousarray(B), x64), np.abs(B) @ np.abs(x64), TOL[dtype],
                     "%s %s trans=%s" % (dtype, layout, trans))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_gemv_16384_every_output(dtype):
    """The benchmark's 16384 x 16384 matrices: y = A x and y = A^T x for the
    row-major and the column-major copy of the same matrix, plain and
    compensated, every output against the oracle.  The column-major copy's
    storage is A^T row-major, so it is downloaded as the oracle's A^T."""
    from paper_1409_0669_amd import ops
    m = n = 16384
    A = W.device_draw(m * n, dtype, 0, 301).view(m, n)
    x = W.device_draw(n, dtype, 0, 401)
    A_col = A.t().contiguous().t()
    x64 = host(x)
    ref = {}
    for trans, B in ((False, host(A)), (True, host(A_col.t()))):
        ref[trans] = (oracle.gemv(B, x64), np.abs(B) @ np.abs(x64))
        del B
    for layout, Ad in (("row", A), ("col", A_col)):
        for trans in (False, True):
            for acc in ("plain", "compensated"):
                y = host(ops.gemv(Ad, x, trans=trans, acc=acc))
                check_vector(y, ref[trans][0], ref[trans][1], TOL[dtype],
                             "%s %s trans=%s %s" % (dtype, layout, trans, acc), plain_f32=plain_reduced(dtype, acc))


def test_composite_cg_step_and_gemv_dot():
    """CG-like step at n = 2^24 and q = A p, <p, q> with A 8192 x 8192, all
    float64 with standard normal entries."""
    from paper_1409_0669_amd import composite
    n = 1 << 24
    a = float(W.uniform(1, 0, 9)[0])
    vals = {k: W.device_draw(n, "f64", 0, 600 + i, dist="normal") for i, k in enumerate("xprq")}
    h = {k: host(v) for k, v in vals.items()}
    x1, r1 = vals["x"].clone(), vals["r"].clone()
    rr = float(composite.cg_step(a, x1, vals["p"], r1, vals["q"]).item())
    xr = oracle.axpby("f64", a, h["p"], 1.0, h["x"])
    rref = oracle.axpby("f64", -a, h["q"], 1.0, h["r"])
    assert bitwise_equal(host(x1), xr)
    assert bitwise_equal(host(r1), rref)
    rr_ref = oracle.dot(rref, rref)
    check_scalar(rr, rr_ref, 0.0, TOL["f64"], "rr")
    x2, r2 = vals["x"].clone(), vals["r"].clone()
    rr2 = float(composite.cg_step_fused(a, x2, vals["p"], r2, vals["q"]).item())
    assert bitwise_equal(host(x2), xr)
    assert bitwise_equal(host(r2), rref)
    check_scalar(rr2, rr_ref, 0.0, TOL["f64"], "rr fused")
    del vals, h, x1, r1, x2, r2
    m = 8192
    A = W.device_draw(m * m, "f64", 0, 700, dist="normal").view(m, m)
    p = W.device_draw(m, "f64", 0, 701, dist="normal")
    A64, p64 = host(A), host(p)
    qref, pqref = oracle.gemv_dot("f64", A64, p64, p64)
    scale = np.abs(A64) @ np.abs(p64)
    # each stored q_i is within tol scale_i of the oracle's, and the reduction
    # adds at most tol sum |p_i q_i|: bound 2 tol sum_i |p_i| scale_i
    bound = 2.0 * float(np.abs(p64) @ scale)
    q, pq = composite.gemv_dot(A, p)
    check_vector(host(q), qref, scale, TOL["f64"], "q")
    check_scalar(float(pq.item()), pqref, bound, TOL["f64"], "pq")
    q2, pq2 = composite.gemv_dot_fused(A, p)
    assert bitwise_equal(host(q2), host(q))
    check_scalar(float(pq2.item()), pqref, bound, TOL["f64"], "pq fused")


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_reduced_precision_compensated_vs_plain(dtype):
    """bf16/f32 storage, float32 accumulation: compensated sums meet the 1e-5
    criterion on the quantised values and are far closer than plain sums; the
    float64 result of the same data is reported against the unquantised
    draws for context."""
    from paper_1409_0669_amd import ops
    n = 1 << 26
    x = W.device_draw(n, dtype, 0, 800)
    y = W.device_draw(n, dtype, 0, 801)
    x64, y64 = host(x), host(y)
    ref = oracle.dot(x64, y64)
    comp = float(ops.dot(x, y, acc="compensated").item())
    plain = float(ops.dot(x, y, acc="plain").item())
    check_scalar(comp, ref, 0.0, TOL[dtype], "compensated")
    check_scalar(plain, ref, 0.0, TOL[dtype], "plain")
    assert abs(comp - ref) <= abs(plain - ref) + 1e-6 * abs(ref)
    m = n_ = 16384 if dtype == "f32" else 8192
    A = W.device_draw(m * n_, dtype, 0, 802).view(m, n_)
    v = W.device_draw(n_, dtype, 0, 803)
    yv = host(ops.gemv(A, v, acc="compensated"))
    A64, v64 = host(A), host(v)
    check_vector(yv, oracle.gemv(A64, v64), np.abs(A64) @ np.abs(v64), TOL[dtype], "gemv comp")


def test_gemv_beyond_int32_elements():
    """A 46341 x 46341 float32 matrix has more elements than a 32-bit index
    holds (2 147 488 281 > 2^31 - 1): y = A x (rows kernel) and y = A^T x
    (cols kernel on the same bytes) on sampled outputs, including the last
    row and column, against the oracle on those rows and columns."""
    from paper_1409_0669_amd import ops
    m = 46341
    A = W.device_draw(m * m, "f32", 0, 710).view(m, m)
    x = W.device_draw(m, "f32", 0, 711)
    x64 = host(x)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, 1, m // 2, m - 2, m - 1], rng.integers(0, m, 12)]))
    for acc in ("plain", "compensated"):
        y = host(ops.gemv(A, x, acc=acc))
        rows = np.stack([host(A[int(i)]) for i in idx])
        check_vector(y[idx], oracle.gemv(rows, x64), np.abs(rows) @ np.abs(x64), TOL["f32"], "rows " + acc)
        yt = host(ops.gemv(A, x, trans=True, acc=acc))
        cols = np.stack([host(A[:, int(j)].contiguous()) for j in idx])
        check_vector(yt[idx], oracle.gemv(cols, x64), np.abs(cols) @ np.abs(x64), TOL["f32"], "cols " + acc)
    del A


def test_ger_beyond_int32_elements():
    """The rank-1 overwrite A = u v^T on 46341 x 46341 float32 entries (more
    than a 32-bit index holds), row-major and then column-major over the same
    bytes: sampled rows and columns, the last ones included, bitwise against
    the oracle's once-rounded products."""
    from paper_1409_0669_amd import ops
    m = 46341
    u = W.device_draw(m, "f32", 0, 720)
    v = W.device_draw(m, "f32", 0, 721)
    u64, v64 = host(u), host(v)
    rng = np.random.default_rng(6)
    idx = np.unique(np.concatenate([[0, 1, m // 2, m - 2, m - 1], rng.integers(0, m, 12)]))
    A = torch.full((m, m), float("nan"), dtype=torch.float32, device="cuda")
    for layout in ("row", "col"):
        view = A if layout == "row" else A.t()    # the transpose of a contiguous A is column-major
        ops.ger(u, v, view)
        for i in idx:
            i = int(i)
            assert bitwise_equal(host(view[i]), oracle.ger("f32", u64[i:i + 1], v64)), (layout, "row", i)
            assert bitwise_equal(host(view[:, i]), oracle.ger("f32", u64, v64[i:i + 1])), (layout, "col", i)
    del A


@pytest.mark.parametrize("acc", ["plain", "compensated"])
def test_batch_beyond_int32_elements(acc):
    """One batch plan holding a 46341 x 46341 float32 GEMV and a dot of
    2^31 + 37 elements (both past a 32-bit index) beside small uneven
    problems: the GEMV on sampled outputs against the oracle on those rows,
    the long dot <1, 1> against its closed form (every chunk partial is an
    exact count and the chunk combine is exact), the small problems in
    full."""
    from paper_1409_0669_amd.batch import BatchPlan
    from tests.batch_util import check, from_sizes
    m, nd = 46341, (1 << 31) + 37
    A = W.device_draw(m * m, "f32", 0, 730).view(m, m)
    x = W.device_draw(m, "f32", 0, 731)
    ones = torch.ones(nd, dtype=torch.float32, device="cuda")
    y = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    guards = []
    gemvs, dots = from_sizes("f32", np.array([37, 300, 5]), np.array([1000, 64, 3000]),
                             np.array([5000, 70000, 1]), seed=7, guards=guards, od=torch.float64)
    plan = BatchPlan(gemvs + [(A, x, y)], dots + [(ones, ones, out)], acc=acc, out_dtype=torch.float64)
    plan.run()
    torch.cuda.synchronize()
    check("f32", acc, gemvs, dots)
    for g in guards:
        g()
    assert float(out.item()) == nd
    x64, yh = host(x), host(y)
    rng = np.random.default_rng(8)
    idx = np.unique(np.concatenate([[0, 1, m // 2, m - 2, m - 1], rng.integers(0, m, 12)]))
    rows = np.stack([host(A[int(i)]) for i in idx])
    check_vector(yh[idx], oracle.gemv(rows, x64), np.abs(rows) @ np.abs(x64), TOL["f32"], "gemv " + acc,
                 plain_f32=plain_reduced("f32", acc))
    assert np.all(np.isfinite(yh))
    plan.close()
    del A, ones


def test_strided_beyond_int32_offsets():
    """Increments that carry element offsets past a 32-bit index: n = 2^30 + 3
    logical elements at increments 2 and -2 span 2^31 + 5 stored elements.
    The strided dot of ones against its closed form n (float64 output: the
    per-thread partials are exact counts and their combine is exact), and a
    strided axpby into increment -2 checked bitwise on sampled logical
    indices, the first and last included."""
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    n = (1 << 30) + 3
    span = 2 * (n - 1) + 1
    ws = ops._ws_ptr(ops.workspace(ops.workspace_size(L.OP_DOT, torch.float32, n=n), torch.device("cuda")))
    ones = torch.ones(span, dtype=torch.float32, device="cuda")
    out = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
    for acc in (L.ACC_PLAIN, L.ACC_COMPENSATED):
        L.check(L.lib.bwla_dot_strided(L.F32, acc, n, ones.data_ptr(), 2, ones.data_ptr(), -2, L.F64,
                                       out.data_ptr(), *ws, ops._stream()))
        assert float(out.item()) == n, acc
    del ones
    y = W.device_draw(span, "f32", 0, 740)
    z = W.device_draw(n, "f32", 0, 741)
    x = torch.full((span,), float("nan"), dtype=torch.float32, device="cuda")
    a, b = 0.75, -1.25
    L.check(L.lib.bwla_axpby_strided(L.F32, n, a, None, y.data_ptr(), 2, b, None, z.data_ptr(), 1, x.data_ptr(), -2,
                                     ops._stream()))
    rng = np.random.default_rng(9)
    i = np.unique(np.concatenate([[0, 1, n // 2, n - 2, n - 1], rng.integers(0, n, 4096)]))
    ti = torch.from_numpy(i).cuda()
    ys, zs, xs = host(y[2 * ti]), host(z[ti]), host(x[2 * (n - 1 - ti)])
    ref = oracle.axpby("f32", oracle.scalar("f32", a), ys, oracle.scalar("f32", b), zs)
    assert bitwise_equal(xs, ref)
    # the gaps between the strided outputs are untouched
    gaps = host(x[2 * torch.from_numpy(np.unique(np.minimum(i, n - 2))).cuda() + 1])
    assert np.all(np.isnan(gaps))


@pytest.mark.parametrize("acc", ["plain", "compensated"])
def test_cg_update_beyond_int32_elements(acc):
    """The fused update x += a p, r -= a q, <r, r> on bf16 vectors of
    2^31 + 37 elements: x and p drawn at random and x checked bitwise on
    sampled indices (the tail included); r = 2, q = 1 and a = 1 make every
    updated r_i exactly 1, so <r, r> is the count n (float64 output; exact
    counts throughout)."""
    from paper_1409_0669_amd import ops
    n = (1 << 31) + 37
    x = W.device_draw(n, "bf16", 0, 750)
    p = W.device_draw(n, "bf16", 0, 751)
    r = torch.full((n,), 2.0, dtype=torch.bfloat16, device="cuda")
    q = torch.ones(n, dtype=torch.bfloat16, device="cuda")
    rng = np.random.default_rng(10 + (acc == "compensated"))
    idx = np.unique(np.concatenate([np.arange(8), rng.integers(0, n, 4096), np.arange(n - 64, n)]))
    ti = torch.from_numpy(idx).cuda()
    x0, p0 = host(x[ti]), host(p[ti])
    rr = float(ops.cg_update(1.0, x, p, r, q, acc=acc, out_dtype=torch.float64).item())
    assert rr == n
    ae = oracle.scalar("bf16", 1.0)
    assert bitwise_equal(host(x[ti]), oracle.axpby("bf16", ae, p0, 1.0, x0))
    assert bitwise_equal(host(r[ti]), np.ones(idx.size))
    del x, p, r, q


@pytest.mark.parametrize("lda", [(1 << 31) + 64, (1 << 31) + 7])
def test_gemv_leading_dimension_beyond_int32(lda):
    """Three rows of 1000 float32 entries lda = 2^31 + 64 (16-byte packs) or
    2^31 + 7 (one element per access) apart: row offsets pass a 32-bit
    index.  y = A x (rows kernel) and y = A^T v (cols kernel) on every output
    against the oracle."""
    from paper_1409_0669_amd import ops
    m, n = 3, 1000
    buf = torch.full(((m - 1) * lda + n,), float("nan"), dtype=torch.float32, device="cuda")
    A = buf.as_strided((m, n), (lda, 1))
    A.copy_(W.device_draw(m * n, "f32", 0, 760).view(m, n))
    x = W.device_draw(n, "f32", 0, 761)
    v = W.device_draw(m, "f32", 0, 762)
    A64 = np.stack([host(A[i]) for i in range(m)])
    x64, v64 = host(x), host(v)
    for acc in ("plain", "compensated"):
        check_vector(host(ops.gemv(A, x, acc=acc)), oracle.gemv(A64, x64), np.abs(A64) @ np.abs(x64), TOL["f32"],
                     "rows " + acc, plain_f32=plain_reduced("f32", acc))
        At = np.ascontiguousarray(A64.T)
        check_vector(host(ops.gemv(A, v, trans=True, acc=acc)), oracle.gemv(At, v64), np.abs(At) @ np.abs(v64),
                     TOL["f32"], "cols " + acc, plain_f32=plain_reduced("f32", acc))
    del buf, A
