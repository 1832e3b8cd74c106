"""Acceptance criteria of the parity tests (test helper).

* Single-rounding operations (copy, scaled addition, rank-1 overwrite, dot
  backward): bitwise equal to the oracle (0 ULP) in matching precision.
* Reductions: many results are correct (the summation order is free), so they
  are compared within a tolerance: 1e-12 for float64 storage, 1e-5 for float32
  and bfloat16 storage (bf16 inputs compared on their quantised values).
  "Relative" is read as condition-scaled, the same for an inner product and
  for each output of a GEMV (a one-row GEMV is an inner product):
  - dot: |got - ref| <= tol * sum |x_i y_i| (for well-conditioned data this
    is close to tol * |ref|; for ill-conditioned sums no float32-accumulated
    order can meet tol * |ref|, compensated summation aside);
  - nrm2: |got - ref| <= tol * |ref| (sum x_i^2 has no cancellation);
  - GEMV: per output, |got_i - ref_i| <= tol * (|A| |x|)_i, and, for a
    product with at least NORMWISE_MIN_OUTPUTS outputs, max |got - ref| <=
    tol * max |ref|.  With fewer outputs max |ref| can be one output that
    cancels, and the normwise check would become the relative error of an
    ill-conditioned inner product, which the inner-product reading above
    rules out (one output per row: a one-row GEMV is an inner product).
  - GEMV followed by <w, y> (fused or not): |got - ref| <= 2 tol *
    sum_i |w_i| (|A| |x|)_i, the GEMV bound carried through w plus the
    inner product's own bound (sum |w_i y_i| is no larger).
"""
from __future__ import annotations

import math

import numpy as np

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5}
NORMWISE_MIN_OUTPUTS = 64


def check_scalar(got: float, ref: float, absum: float, tol: float, what: str = "") -> None:
    """absum = sum |x_i y_i| for an inner product (condition scale); 0 when the
    scale is |ref| itself (norms, sums without cancellation)."""
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


def check_vector(got: np.ndarray, ref: np.ndarray, scale: np.ndarray, tol: float, what: str = "") -> None:
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
    if rmax > 0 and ref.size >= NORMWISE_MIN_OUTPUTS:
        assert float(err.max()) <= tol * rmax, "%s: normwise err %.3e" % (what, float(err.max()) / rmax)


def bitwise_equal(got: np.ndarray, ref: np.ndarray) -> bool:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return got.shape == ref.shape and bool(np.all((got == ref) | (np.isnan(got) & np.isnan(ref))))
