"""Acceptance criteria of the parity tests (test helper).

* Single-rounding operations (copy, scaled addition, rank-1 overwrite, dot
  backward): bitwise equal to the oracle (0 ULP) in matching precision.
* Reductions: many results are correct (the summation order is free), so they
  are compared within a tolerance: 1e-12 for float64 storage, 1e-5 for float32
  and bfloat16 storage (bf16 inputs compared on their quantised values).
  "Relative" is relative to the exact result, |got - ref| <= tol * |ref|, for
  every reduction with float64 storage and for every compensated one (these
  carry, or add up in, at least float64 precision).  The one exception is
  the PLAIN float32 accumulation of float32 and bfloat16 data, whose rounding
  error is of order u_f32 * sum |terms| however the sum is ordered: for an
  ill-conditioned inner product (|ref| << sum |x_i y_i|) no float32-accumulated
  order meets tol * |ref|, so there the bound is condition-scaled, tol *
  max(|ref|, sum |x_i y_i|) (``cond_scale``).  The measured case: one dot of
  the uneven batch with |ref| = 0.44 and sum |x_i y_i| = 14914, plain f32
  error 2.8e-5 * |ref| (8e-10 of the condition scale); the compensated mode
  met 1e-5 * |ref| there.
  - nrm2 and asum: |got - ref| <= tol * |ref| (no cancellation).
  - GEMV: per output, |got_i - ref_i| <= tol * (|A| |x|)_i (the componentwise
    condition scale: a per-output relative bound fails on outputs that cancel
    to near zero), and normwise max |got - ref| <= tol * max |ref|.  The
    normwise check is dropped only for a PLAIN float32-accumulated product
    with fewer than NORMWISE_MIN_OUTPUTS outputs: max |ref| can then be one
    output that cancels, and the check would become the relative error of an
    ill-conditioned float32 inner product, excluded above.  (The measured
    case: a one-row plain bf16 GEMV of the randomised sweep, relative error
    1.085e-5, within its condition-scaled bound.)
  - GEMV followed by <w, y> (fused or not): |got - ref| <= 2 tol *
    sum_i |w_i| (|A| |x|)_i, the GEMV bound carried through w plus the
    inner product's own bound (sum |w_i y_i| is no larger).
"""
from __future__ import annotations

import math

import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5}
NORMWISE_MIN_OUTPUTS = 64


def plain_reduced(dtype, acc) -> bool:
    """True for plain float32 accumulation of float32 or bfloat16 data (acc
    "plain" or 0), the one case judged on the condition scale."""
    return dtype in ("f32", "bf16") and acc in ("plain", 0)


def cond_scale(dtype, acc, absum: float) -> float:
    """The ``absum`` argument of :func:`check_scalar` for an inner product:
    sum |x_i y_i| for plain float32 accumulation of f32/bf16 data, else 0
    (the bound is then tol * |ref|)."""
    return float(absum) if plain_reduced(dtype, acc) else 0.0


def check_scalar(got: float, ref: float, absum: float, tol: float, what: str = "") -> None:
    """Asserts |got - ref| <= tol * max(|ref|, absum).  absum is 0 for the
    relative bound (every reduction but the plain float32-accumulated inner
    product, see ``cond_scale``); a derived absolute scale otherwise."""
    if not math.isfinite(ref):  # an infinite or NaN sum is reproduced exactly
        assert got == ref or (math.isnan(got) and math.isnan(ref)), "%s: got %r for %r" % (what, got, ref)
        return
    err = abs(got - ref)
    scale = max(abs(ref), absum)
    if scale == 0.0:
        assert got == 0.0, "%s: got %r for an exact zero" % (what, got)
        return
    assert err <= tol * scale, "%s: err %.3e > %.1e x scale %.3e (got %r ref %r)" % (
        what, err, tol, scale, got, ref)


def check_vector(got: np.ndarray, ref: np.ndarray, scale: np.ndarray, tol: float, what: str = "",
                 plain_f32: bool = False) -> None:
    """GEMV criterion: componentwise against ``scale`` = |A| |x|, and normwise
    against max |ref| -- skipped for fewer than NORMWISE_MIN_OUTPUTS outputs
    only when ``plain_f32`` (plain float32 accumulation, see
    ``plain_reduced``)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    if ref.size == 0:
        return
    err = np.abs(got - ref)
    bad = err > tol * np.maximum(scale, 1e-300)
    assert not bad.any(), "%s: %d entries beyond componentwise tol %.1e; worst %.3e at %d" % (
        what, int(bad.sum()), tol, float((err / np.maximum(scale, 1e-300)).max()),
        int(np.argmax(err / np.maximum(scale, 1e-300))))
    rmax = float(np.abs(ref).max())
    if rmax > 0 and (ref.size >= NORMWISE_MIN_OUTPUTS or not plain_f32):
        assert float(err.max()) <= tol * rmax, "%s: normwise err %.3e" % (what, float(err.max()) / rmax)


def bitwise_equal(got: np.ndarray, ref: np.ndarray) -> bool:
    """Same value and same sign bit in every entry (so -0 differs from +0);
    any NaN equals any NaN (payloads are not compared)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.shape != ref.shape:
        return False
    same = (got == ref) & (np.signbit(got) == np.signbit(ref))
    return bool(np.all(same | (np.isnan(got) & np.isnan(ref))))
