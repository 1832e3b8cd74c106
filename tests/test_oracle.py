"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something other than itself: exact rational
arithmetic (correctly rounded with ``tests/exact.py``), closed forms, special
cases that reduce to another operation, invariants, or the published error bound
of the Dot2 algorithm.  The cases are chosen so that a plausible slip in the
oracle (a dropped compensation term, a swapped stride, a transposed operand, a
double rounding) makes one of them fail.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W
from tests.exact import dot2_bound, exact_dot, exact_dot_int, rn

PRECS = ("f64", "f32", "bf16")


def _vals(prec, n, stream, seed=7):
    s, x = W.vector(n, prec, seed=seed, stream=stream)
    return x


# --------------------------------------------------------------------------
# rounding to bf16
# --------------------------------------------------------------------------

def test_bf16_rounding_matches_exact_nearest_even():
    rng = np.random.default_rng(1)
    # random f32 values over many binades, plus exact ties and near-ties
    vals = list(rng.standard_normal(2000).astype(np.float32) * np.float32(2.0) ** rng.integers(-20, 20, 2000).astype(np.float32))
    for k in range(1, 300):
        base = np.float32(1.0 + k / 128.0)            # exactly representable in bf16 when k < 128
        half_ulp = np.float32(2.0 ** -8)
        vals += [base + half_ulp, base - half_ulp, base + half_ulp * np.float32(1.0000001),
                 -(base + half_ulp)]
    for v in vals:
        v = float(np.float32(v))
        got = oracle.round_bf16(v)
        assert Fraction(got) == rn(Fraction(v), "bf16"), v


def test_bf16_rounding_special_values():
    assert oracle.round_bf16(0.0) == 0.0
    assert math.copysign(1.0, oracle.round_bf16(-0.0)) == -1.0
    assert oracle.round_bf16(float("inf")) == float("inf")
    assert math.isnan(oracle.round_bf16(float("nan")))
    fmax = float(np.finfo(np.float32).max)
    assert oracle.round_bf16(fmax) == float("inf")       # rounds past the largest bf16
    # ties go to the even neighbour: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert oracle.round_bf16(1.0 + 2.0 ** -8) == 1.0
    assert oracle.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2 * 2.0 ** -7


# --------------------------------------------------------------------------
# scaled vector addition x <- alpha y + beta z
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", PRECS)
def test_axpby_matches_exact_rounding_sequence(prec):
    n = 600
    y, z = _vals(prec, n, 1), _vals(prec, n, 2)
    comp = "f64" if prec == "f64" else "f32"
    alpha = oracle.scalar(prec, 0.7312345678901234)
    beta = oracle.scalar(prec, -1.2345678901234567)
    assert Fraction(alpha) == rn(Fraction(0.7312345678901234), comp)
    x = oracle.axpby(prec, alpha, y, beta, z)
    for i in range(n):
        bz = rn(Fraction(beta) * Fraction(z[i]), comp)
        r = rn(Fraction(alpha) * Fraction(y[i]) + bz, comp)
        if prec == "bf16":
            r = rn(r, "bf16")
        assert Fraction(x[i]) == r, (i, x[i], float(r))


@pytest.mark.parametrize("prec", PRECS)
def test_axpby_special_cases(prec):
    n = 1000
    y, z = _vals(prec, n, 3), _vals(prec, n, 4)
    # alpha = 1, beta = 0 reduces to a copy
    assert np.array_equal(oracle.axpby(prec, 1.0, y, 0.0, z), oracle.copy(y))
    # powers of two: both products are exact, so the result is the sum
    # rounded once in the compute precision (numpy's own float32/float64 add)
    if prec != "bf16":
        ft = np.float64 if prec == "f64" else np.float32
        x = oracle.axpby(prec, 0.5, y, -4.0, z)
        assert np.array_equal(x, (ft(0.5) * y.astype(ft) - ft(4.0) * z.astype(ft)).astype(np.float64))
        # alpha = -1, beta = 1 with y == z cancels exactly
        assert np.all(oracle.axpby(prec, -1.0, y, 1.0, y) == 0.0)
        # scaling by 2 then by 1/2 returns the input (exact power-of-two scaling)
        x2 = oracle.axpby(prec, 2.0, y, 0.0, z)
        assert np.array_equal(oracle.axpby(prec, 0.5, x2, 0.0, z), y)
    # beta = 1: one rounding of alpha*y + z (fused multiply-add)
    a = oracle.scalar(prec, 0.3)
    comp = "f64" if prec == "f64" else "f32"
    x = oracle.axpby(prec, a, y, 1.0, z)
    for i in range(0, n, 37):
        r = rn(Fraction(a) * Fraction(y[i]) + Fraction(z[i]), comp)
        if prec == "bf16":
            r = rn(r, "bf16")
        assert Fraction(x[i]) == r


def test_axpby_is_not_double_rounded_in_f32():
    # a case where computing in double and rounding to f32 once differs from
    # the f32 sequence RN(alpha*y + RN(beta*z)): beta*z has bits below f32
    y = np.array([1.0])
    z = np.array([float(np.float32(1.0 + 2.0 ** -23))])
    alpha, beta = 1.0, float(np.float32(1.0 + 2.0 ** -23))
    x = oracle.axpby("f32", alpha, y, beta, z)[0]
    bz = rn(Fraction(beta) * Fraction(z[0]), "f32")
    assert Fraction(x) == rn(Fraction(1) + bz, "f32")


def test_scalar_with_device_factor():
    assert oracle.scalar("f64", 3.0, 0.1) == 3.0 * 0.1
    h, d = 0.1, 0.3
    assert Fraction(oracle.scalar("f32", h, d)) == rn(rn(Fraction(h), "f32") * rn(Fraction(d), "f32"), "f32")
    assert oracle.scalar("bf16", 2.0) == 2.0


# --------------------------------------------------------------------------
# inner product
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 200, 1000])
def test_dot_within_dot2_bound_of_exact(n):
    x, y = _vals("f64", n, 10 + n), _vals("f64", n, 20 + n)
    s = exact_dot(x, y)
    absum = sum(abs(Fraction(float(a)) * Fraction(float(b))) for a, b in zip(x, y))
    r = oracle.dot(x, y)
    assert abs(Fraction(r) - s) <= Fraction(dot2_bound(n, s, absum))
    # for these well-conditioned sums the result is the correctly rounded one
    assert r == float(s)


def test_dot_long_vector_correctly_rounded():
    n = 1 << 16
    x, y = _vals("f64", n, 31), _vals("f64", n, 32)
    s = exact_dot_int(x, y)
    assert oracle.dot(x, y) == float(s)


def test_dot_ill_conditioned_needs_compensation():
    # plain summation loses the small terms entirely; the exact value is 3
    x = np.array([2.0 ** 60, 1.0, -(2.0 ** 60), 2.0, 2.0 ** 55, -(2.0 ** 55)])
    y = np.ones_like(x)
    assert oracle.dot(x, y) == 3.0
    assert float(np.sum(x)) != 3.0
    # product errors matter too: (1 + 2^-30)^2 - 1 - 2^-29 = 2^-60 exactly
    a = 1.0 + 2.0 ** -30
    x = np.array([a, -1.0, -(2.0 ** -29)])
    y = np.array([a, 1.0, 1.0])
    assert oracle.dot(x, y) == 2.0 ** -60


def test_dot_generated_ill_conditioned_random():
    rng = np.random.default_rng(5)
    for trial in range(20):
        n = 50
        big = rng.uniform(-1, 1, n // 2) * 2.0 ** rng.integers(20, 60, n // 2)
        x = np.concatenate([big, -big, rng.uniform(-1, 1, 6)])
        y = np.ones_like(x)
        perm = rng.permutation(x.size)
        x, y = x[perm], y[perm]
        s = exact_dot(x, y)
        absum = sum(abs(Fraction(float(v))) for v in x)
        r = oracle.dot(x, y)
        assert abs(Fraction(r) - s) <= Fraction(dot2_bound(x.size, s, absum))


@pytest.mark.parametrize("n", [1, 100, 12345, 1 << 20])
def test_dot_closed_forms(n):
    ones = np.ones(n)
    assert oracle.dot(ones, ones) == n
    i = np.arange(n, dtype=np.float64)
    assert oracle.dot(i, ones) == n * (n - 1) // 2
    if n <= 12345:
        assert oracle.dot(i, i) == (n - 1) * n * (2 * n - 1) // 6
    alt = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    assert oracle.dot(alt, ones) == (n % 2)


def test_dot_and_nrm2_with_infinite_and_nan_entries():
    """The IEEE value of a sum with an infinite term is that infinity (NaN
    for inf - inf or a NaN term); the compensation terms must not turn it
    into NaN."""
    x = np.array([1.0, np.inf, 2.0])
    y = np.array([3.0, 1.0, -1.0])
    assert oracle.dot(x, y) == np.inf
    assert oracle.dot(x, -y) == -np.inf
    assert oracle.nrm2(x) == np.inf
    assert np.isnan(oracle.dot(np.array([np.inf, -np.inf]), np.ones(2)))
    assert np.isnan(oracle.dot(np.array([1.0, np.nan]), np.ones(2)))
    assert oracle.dot(np.array([1e300, 1e300]), np.array([1e10, 1e10])) == np.inf  # overflow


def test_dot_empty_and_strided():
    assert oracle.dot([], []) == 0.0
    lib = oracle._load()
    x = np.arange(12, dtype=np.float64)
    y = np.ones(12)
    # stride 3 over x picks 0, 3, 6, 9
    r = lib.o_dot(4, oracle._ptr(x), 3, oracle._ptr(y), 1)
    assert r == 18.0


def test_dot_order_invariance_within_bound():
    n = 5000
    x, y = _vals("f32", n, 41), _vals("f32", n, 42)
    rng = np.random.default_rng(3)
    p = rng.permutation(n)
    r1, r2 = oracle.dot(x, y), oracle.dot(x[p], y[p])
    s = exact_dot(x, y)
    # bf16/f32 products are exact in f64, so Dot2 is correctly rounded here
    assert r1 == r2 == float(s)


# --------------------------------------------------------------------------
# norm
# --------------------------------------------------------------------------

def test_nrm2_closed_forms():
    assert oracle.nrm2([3.0, 4.0]) == 5.0
    assert oracle.nrm2([0.0, -12.0, 5.0]) == 13.0
    for n, c in [(1, 0.5), (4, 2.0), (10000, 0.25), (1 << 20, -8.0)]:
        assert oracle.nrm2(np.full(n, c)) == abs(c) * math.isqrt(n)
    e = np.zeros(1000)
    e[417] = -0.123
    assert oracle.nrm2(e) == 0.123
    assert oracle.nrm2([]) == 0.0


def test_nrm2_random_correctly_rounded_sqrt():
    x = _vals("f64", 3000, 51)
    s = exact_dot(x, x)
    # sqrt of the correctly rounded sum, itself correctly rounded
    assert oracle.nrm2(x) == math.sqrt(float(s))


# --------------------------------------------------------------------------
# matrix-vector product
# --------------------------------------------------------------------------

LAYOUTS = (oracle.ROW_MAJOR, oracle.COL_MAJOR)


def _flat(A, layout, pad=0):
    m, n = A.shape
    if layout == oracle.ROW_MAJOR:
        lda = n + pad
        buf = np.full((m, lda), np.nan)
        buf[:, :n] = A
    else:
        lda = m + pad
        buf = np.full((n, lda), np.nan)
        buf[:, :m] = A.T
    return buf.reshape(-1), lda


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("shape", [(8, 8), (5, 7), (7, 3), (1, 6), (6, 1)])
def test_gemv_exact_small(layout, trans, shape):
    m, n = shape
    rng = np.random.default_rng(m * 10 + n)
    A = rng.uniform(-1, 1, (m, n))
    x = rng.uniform(-1, 1, m if trans else n)
    flat, lda = _flat(A, layout, pad=3)
    y = oracle.gemv(flat, x, layout=layout, trans=trans, m=m, n=n, lda=lda)
    B = A.T if trans else A
    for i in range(B.shape[0]):
        assert y[i] == float(exact_dot(B[i], x)), (i,)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_gemv_identity_and_permutation(layout):
    n = 50
    x = _vals("f64", n, 61)
    I = np.eye(n)
    assert np.array_equal(oracle.gemv(I, x, layout=layout), x)
    perm = np.random.default_rng(2).permutation(n)
    P = np.eye(n)[perm]
    assert np.array_equal(oracle.gemv(P, x, layout=layout), x[perm])
    assert np.array_equal(oracle.gemv(P, x, layout=layout, trans=1), x[np.argsort(perm)])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_gemv_rank_one_small_integers(layout):
    rng = np.random.default_rng(8)
    u = rng.integers(-9, 10, 37).astype(np.float64)
    v = rng.integers(-9, 10, 23).astype(np.float64)
    x = rng.integers(-9, 10, 23).astype(np.float64)
    A = np.outer(u, v)
    assert np.array_equal(oracle.gemv(A, x, layout=layout), u * float(v @ x))
    xt = rng.integers(-9, 10, 37).astype(np.float64)
    assert np.array_equal(oracle.gemv(A, xt, layout=layout, trans=1), v * float(u @ xt))


def test_gemv_reduces_to_dot_and_scaling():
    x = _vals("f64", 300, 71)
    a = _vals("f64", 300, 72)
    assert oracle.gemv(a.reshape(1, -1), x)[0] == oracle.dot(a, x)
    col = _vals("f64", 40, 73)
    x0 = np.array([0.3])
    assert np.array_equal(oracle.gemv(col.reshape(-1, 1), x0), col * 0.3)


def test_gemv_layout_swap_identity():
    rng = np.random.default_rng(9)
    A = rng.uniform(-1, 1, (30, 20))
    x = rng.uniform(-1, 1, 20)
    row_buf = A.reshape(-1)            # row-major A == column-major A^T
    y1 = oracle.gemv(row_buf, x, layout=oracle.ROW_MAJOR, trans=0, m=30, n=20, lda=20)
    y2 = oracle.gemv(row_buf, x, layout=oracle.COL_MAJOR, trans=1, m=20, n=30, lda=20)
    assert np.array_equal(y1, y2)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("trans", [0, 1])
def test_gemv_dot_f64_exact(layout, trans):
    """y_i is the correctly rounded row product and s is within the Dot2
    bound of the exact <w, y> (y as stored), computed with rationals."""
    m, n = 9, 13
    rng = np.random.default_rng(31 + trans)
    A = rng.uniform(-1, 1, (m, n))
    x = rng.uniform(-1, 1, m if trans else n)
    w = rng.uniform(-1, 1, n if trans else m)
    flat, lda = _flat(A, layout, pad=2)
    y, s = oracle.gemv_dot("f64", flat, x, w, layout=layout, trans=trans, m=m, n=n, lda=lda)
    B = A.T if trans else A
    for i in range(B.shape[0]):
        assert y[i] == float(exact_dot(B[i], x)), i
    ex = exact_dot(w, y)
    absum = sum(abs(Fraction(float(a)) * Fraction(float(b))) for a, b in zip(w, y))
    assert abs(Fraction(s) - ex) <= Fraction(dot2_bound(len(w), ex, absum))


def test_gemv_dot_f32_rounds_y_before_the_inner_product():
    """With f32 storage the inner product takes the stored (rounded) y:
    rows (1, 2^-30) and (3, 2^-28) against x = (1, 1) give y = (1, 3) in
    float32, so <w, y> = 1 + 3 = 4, not 4 + 5 * 2^-30."""
    A = np.array([[1.0, 2.0 ** -30], [3.0, 2.0 ** -28]])
    y, s = oracle.gemv_dot("f32", A, np.ones(2), np.ones(2))
    assert y.tolist() == [1.0, 3.0] and s == 4.0
    y, s = oracle.gemv_dot("f64", A, np.ones(2), np.ones(2))
    assert s == 4.0 + 5 * 2.0 ** -30
    # a value halfway between two floats rounds to the even one
    y, _ = oracle.gemv_dot("f32", np.array([[1.0, 2.0 ** -24]]), np.ones(2), np.ones(1))
    assert y[0] == 1.0
    y, _ = oracle.gemv_dot("f32", np.array([[1.0 + 2.0 ** -23, 2.0 ** -24]]), np.ones(2), np.ones(1))
    assert y[0] == 1.0 + 2.0 ** -22


def test_gemv_dot_small_integers_and_quadratic_form():
    """Small integers are exact throughout: y = A x and s = w^T A x; with
    A = I and w = x the result is the squared norm."""
    rng = np.random.default_rng(12)
    A = rng.integers(-6, 7, (40, 30)).astype(np.float64)
    x = rng.integers(-6, 7, 30).astype(np.float64)
    w = rng.integers(-6, 7, 40).astype(np.float64)
    for prec in ("f64", "f32"):
        y, s = oracle.gemv_dot(prec, A, x, w)
        assert y.tolist() == (A @ x).tolist()
        assert s == float(sum(int(a) * int(b) for a, b in zip(w, A @ x)))
    y, s = oracle.gemv_dot("f64", A.T, w, x, layout=oracle.ROW_MAJOR, trans=0)
    y2, s2 = oracle.gemv_dot("f64", A, w, x, trans=1)
    assert y.tolist() == y2.tolist() and s == s2
    _, s = oracle.gemv_dot("f64", np.eye(30), x, x)
    assert s == float(x @ x)
    with pytest.raises(ValueError):
        oracle.gemv_dot("bf16", A, x, w)


def test_gemv_empty():
    assert oracle.gemv(np.zeros((0, 5)), np.ones(5)).size == 0
    assert np.array_equal(oracle.gemv(np.zeros((4, 0)), np.ones(0)), np.zeros(4))


# --------------------------------------------------------------------------
# rank-1 overwrite and adjoints
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("layout", LAYOUTS)
def test_ger_single_rounding(prec, layout):
    m, n = 13, 9
    u, v = _vals(prec, m, 81), _vals(prec, n, 82)
    pad = 2
    lda = (n if layout == oracle.ROW_MAJOR else m) + pad
    A = oracle.ger(prec, u, v, layout=layout, lda=lda)
    for i in range(m):
        for j in range(n):
            at = i * lda + j if layout == oracle.ROW_MAJOR else i + j * lda
            r = Fraction(u[i]) * Fraction(v[j])
            r = rn(r, "f64") if prec == "f64" else rn(rn(r, "f32"), prec)
            assert Fraction(A[at]) == r
    # padding untouched
    lines = m if layout == oracle.ROW_MAJOR else n
    pad_vals = A.reshape(lines, lda)[:, lda - pad:]
    assert np.all(pad_vals == 0.0)


@pytest.mark.parametrize("prec", PRECS)
def test_dot_backward_is_scaling(prec):
    n = 400
    x, y = _vals(prec, n, 91), _vals(prec, n, 92)
    zbar = oracle.scalar(prec, -0.618)
    dx, dy = oracle.dot_backward(prec, zbar, x, y)
    comp = "f64" if prec == "f64" else "f32"
    for i in range(0, n, 7):
        for g, src in ((dx, y), (dy, x)):
            r = rn(Fraction(zbar) * Fraction(src[i]), comp)
            if prec == "bf16":
                r = rn(r, "bf16")
            assert Fraction(g[i]) == r


@pytest.mark.parametrize("prec", PRECS)
def test_dot_backward_ieee_specials(prec):
    """dz/dx_i = y_i exactly, so the gradient entry is one IEEE product: an
    infinite y_i gives an infinity with the sign of zbar * y_i, a NaN stays
    NaN, a zero keeps the sign of the product (-zbar * +0 = -0), and
    zbar = 0 times an infinity is NaN.  A form with an extra 0 * y_i term
    (a scaled addition with beta = 0) fails the first and the signed zeros."""
    y = np.array([np.inf, -np.inf, np.nan, 0.0, -0.0, 1.5, -0.25])
    x = np.array([2.0, -0.0, 0.0, np.inf, np.nan, -4.0, 8.0])
    for zbar, dx_ref, dy_ref in (
            (-2.0, [-np.inf, np.inf, np.nan, -0.0, 0.0, -3.0, 0.5],
             [-4.0, 0.0, -0.0, -np.inf, np.nan, 8.0, -16.0]),
            (0.5, [np.inf, -np.inf, np.nan, 0.0, -0.0, 0.75, -0.125],
             [1.0, -0.0, 0.0, np.inf, np.nan, -2.0, 4.0]),
            (0.0, [np.nan, np.nan, np.nan, 0.0, -0.0, 0.0, -0.0],
             [0.0, -0.0, 0.0, np.nan, np.nan, -0.0, 0.0]),
            (-0.0, [np.nan, np.nan, np.nan, -0.0, 0.0, -0.0, 0.0],
             [-0.0, 0.0, -0.0, np.nan, np.nan, 0.0, -0.0])):
        dx, dy = oracle.dot_backward(prec, oracle.scalar(prec, zbar), x, y)
        for got, ref in ((dx, dx_ref), (dy, dy_ref)):
            for g, r in zip(got, ref):
                if math.isnan(r):
                    assert math.isnan(g), (prec, zbar, got, ref)
                else:
                    assert g == r and math.copysign(1.0, g) == math.copysign(1.0, r), (prec, zbar, got, ref)


@pytest.mark.parametrize("prec", PRECS)
def test_dot_backward_matches_derivative_of_exact_dot(prec):
    """The exact inner product is linear in each x_i with slope y_i (and in
    each y_i with slope x_i): setting the entry to 1 and then to 0 changes
    the exact sum (Fraction arithmetic) by the slope, so the gradient entry
    is zbar times that difference, rounded once."""
    n = 24
    x, y = _vals(prec, n, 93), _vals(prec, n, 94)
    zbar = oracle.scalar(prec, 0.8125)
    dx, dy = oracle.dot_backward(prec, zbar, x, y)
    comp = "f64" if prec == "f64" else "f32"

    def slope_of(a, b, i):
        a1, a0 = a.copy(), a.copy()
        a1[i], a0[i] = 1.0, 0.0
        return exact_dot(a1, b) - exact_dot(a0, b)

    for i in range(n):
        slope_x, slope_y = slope_of(x, y, i), slope_of(y, x, i)
        for g, slope in ((dx[i], slope_x), (dy[i], slope_y)):
            r = rn(Fraction(zbar) * slope, comp)
            if prec == "bf16":
                r = rn(r, "bf16")
            assert Fraction(float(g)) == r


def test_gemv_adjoint_identity_and_finite_differences():
    # <w, A x> is bilinear, so the central difference with h = 1e-6 has no
    # truncation error; what remains is rounding of order u*|L|/h.
    rng = np.random.default_rng(12)
    m, n = 64, 48
    A = rng.uniform(-1, 1, (m, n))
    x = rng.uniform(-1, 1, n)
    w = rng.uniform(-1, 1, m)
    dx, dA = oracle.gemv_backward("f64", A, x, w)
    # adjoint identity <w, A x> == <A^T w, x>
    lhs = oracle.dot(w, oracle.gemv(A, x))
    rhs = oracle.dot(dx, x)
    assert abs(lhs - rhs) <= 1e-13 * np.sum(np.abs(w) @ np.abs(A) * np.abs(x))
    h = 1e-6
    L = lambda AA, xx: oracle.dot(w, oracle.gemv(AA, xx))
    for j in range(0, n, 5):
        e = np.zeros(n)
        e[j] = h
        fd = (L(A, x + e) - L(A, x - e)) / (2 * h)
        assert abs(fd - dx[j]) <= 1e-8 * (1 + abs(fd))
    dA2 = dA.reshape(m, n)
    for (i, j) in [(0, 0), (5, 7), (63, 47), (30, 2)]:
        E = np.zeros((m, n))
        E[i, j] = h
        fd = (L(A + E, x) - L(A - E, x)) / (2 * h)
        assert abs(fd - dA2[i, j]) <= 1e-8 * (1 + abs(fd))


# --------------------------------------------------------------------------
# BLAS-interface additions: increments, scal, asum, alpha/beta GEMV
# --------------------------------------------------------------------------

def test_strided_positions_follow_the_blas_convention():
    """Checked against numpy slicing: a negative increment walks the buffer
    backwards from its end, a zero increment repeats the first entry."""
    buf = np.arange(20, dtype=np.float64) * 1.5
    assert oracle.strided(buf, 10, 2).tolist() == buf[::2][:10].tolist()
    assert oracle.strided(buf, 20, -1).tolist() == buf[::-1].tolist()
    assert oracle.strided(buf, 7, -3).tolist() == buf[::3][:7][::-1].tolist()
    assert oracle.strided(buf, 5, 0).tolist() == [buf[0]] * 5
    assert oracle.strided(buf, 0, 4).size == 0
    for inc in (1, 2, -2, 3):
        n = (20 - 1) // abs(inc) + 1
        v = oracle.strided(buf, n, inc)
        assert oracle.scatter(buf, v, inc).tolist() == buf.tolist()
    out = oracle.scatter(np.zeros(9), np.array([1.0, 2.0, 3.0]), -4)
    assert out.tolist() == [3.0, 0, 0, 0, 2.0, 0, 0, 0, 1.0]


@pytest.mark.parametrize("prec", PRECS)
def test_scal_single_rounding(prec):
    rng = np.random.default_rng(91)
    y = _vals(prec, 300, 92)
    for alpha in (0.7, -3.25, 1e-3):
        a = oracle.scalar(prec, alpha)
        x = oracle.scal(prec, a, y)
        for xi, yi in zip(x, y):
            exact = Fraction(a) * Fraction(float(yi))
            ref = rn(exact, "f64") if prec == "f64" else rn(rn(exact, "f32"), prec)
            assert Fraction(float(xi)) == ref
    del rng


def test_scal_ieee_specials_differ_from_axpby_with_zero_beta():
    y = np.array([np.inf, -np.inf, np.nan, -0.0, 0.0, 1.0])
    x = oracle.scal("f64", 2.0, y)
    assert x[0] == np.inf and x[1] == -np.inf and np.isnan(x[2])
    assert math.copysign(1.0, x[3]) == -1.0 and math.copysign(1.0, x[4]) == 1.0 and x[5] == 2.0
    # axpby with beta = 0 forms 0 * z, which is NaN for an infinite z
    assert np.isnan(oracle.axpby("f64", 2.0, y, 0.0, y)[0])
    assert np.isnan(oracle.scal("f32", 0.0, np.array([np.inf]))[0])  # 0 * inf is NaN


def test_asum_against_fsum_and_special_cases():
    """math.fsum is the correctly rounded sum; Sum2's error is at most
    u |s| + gamma_{n-1}^2 sum |x_i| (Ogita, Rump, Oishi 2005), i.e. about one
    rounding for terms of one sign."""
    rng = np.random.default_rng(93)
    for n in (1, 2, 17, 1000, 100000):
        x = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
        ref = math.fsum(np.abs(x))
        u = 2.0 ** -53
        g = (n - 1) * u / (1 - (n - 1) * u)
        assert abs(oracle.asum(x) - ref) <= u * ref + g * g * ref
    x = rng.integers(-1000, 1000, 5000).astype(np.float64)
    assert oracle.asum(x) == float(np.abs(x).sum())  # integers: exact
    assert oracle.asum(np.array([])) == 0.0
    assert oracle.asum(np.array([-np.inf, 1.0])) == np.inf
    assert np.isnan(oracle.asum(np.array([np.nan, 1.0])))
    # a sum that plain double accumulation gets wrong: 1 + 2^-53 (many times)
    x = np.array([1.0] + [2.0 ** -53] * 1000)
    assert oracle.asum(x) == math.fsum(x) == 1.0 + 1000 * 2.0 ** -53


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("trans", [0, 1])
def test_gemv_axpby_small_integers_exact(layout, trans):
    rng = np.random.default_rng(94 + trans)
    m, n = 11, 7
    A = rng.integers(-5, 6, (m, n)).astype(np.float64)
    x = rng.integers(-5, 6, m if trans else n).astype(np.float64)
    y = rng.integers(-5, 6, n if trans else m).astype(np.float64)
    flat, lda = _flat(A, layout, pad=1)
    B = A.T if trans else A
    for prec in ("f64", "f32"):
        got = oracle.gemv_axpby(prec, 2.0, flat, x, -3.0, y, layout=layout, trans=trans, m=m, n=n, lda=lda)
        assert got.tolist() == (2.0 * (B @ x) - 3.0 * y).tolist()
        # beta == 0: y is not read (a NaN there does not propagate)
        got = oracle.gemv_axpby(prec, -1.5, flat, x, 0.0, np.full(y.size, np.nan), layout=layout,
                                trans=trans, m=m, n=n, lda=lda)
        assert got.tolist() == (-1.5 * (B @ x)).tolist()
    with pytest.raises(ValueError):
        oracle.gemv_axpby("bf16", 1.0, A, x, 0.0, y)


def test_gemv_axpby_rounding_sequence():
    """f32 output: the product is rounded to float32 before the update.
    s = 1 + 2^-30 is stored as 1; then 1 + RN(1 * 2^-24) is a tie that rounds
    to the even 1.  In float64 the terms survive."""
    A = np.array([[1.0, 2.0 ** -30]])
    got = oracle.gemv_axpby("f32", 1.0, A, np.ones(2), 1.0, np.array([2.0 ** -24]))
    assert got.tolist() == [1.0]
    got = oracle.gemv_axpby("f64", 1.0, A, np.ones(2), 1.0, np.array([2.0 ** -24]))
    assert got.tolist() == [1.0 + 2.0 ** -30 + 2.0 ** -24]
    # alpha is rounded to float32 first: 0.1 -> 0x3dcccccd
    a32 = float(np.float32(0.1))
    got = oracle.gemv_axpby("f32", 0.1, np.array([[3.0]]), np.ones(1), 0.0, np.zeros(1))
    assert got[0] == float(np.float32(a32 * 3.0))

