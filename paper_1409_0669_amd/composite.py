"""Composite operations built from the tuned kernels: the paper's point is
that once the copy-like kernels are fast, composite operations built from them
are fast too (abstract; Section 3.4).

* ``cg_step``: the vector part of a conjugate-gradient iteration,
  x += a p; r -= a q; rr = <r, r>, as three library calls (stream-ordered,
  scalars stay on the device), 7 n elements of traffic.
* ``cg_step_fused``: the same step in one pass (6 n elements, one launch plus
  the reduction's second stage); elementwise results are bitwise those of
  ``cg_step``.
* ``gemv_dot``: q = A p followed by <p, q>; ``gemv_dot_fused`` the same with
  the inner product in the GEMV's epilogue.
"""
from __future__ import annotations

import torch

from . import ops


def cg_step(a: float, x, p, r, q, acc="plain", alpha_dev=None):
    ops.axpby(a, p, 1.0, x, out=x, alpha_dev=alpha_dev)
    if alpha_dev is None:
        ops.axpby(-a, q, 1.0, r, out=r)
    else:
        ops.axpby(-a, q, 1.0, r, out=r, alpha_dev=alpha_dev)
    return ops.dot(r, r, acc=acc)


def cg_step_fused(a: float, x, p, r, q, acc="plain", alpha_dev=None):
    return ops.cg_update(a, x, p, r, q, acc=acc, alpha_dev=alpha_dev)


def gemv_dot(A, p, acc="plain", q=None):
    """q = A p and <p, q> as two library calls."""
    q = ops.gemv(A, p, acc=acc, out=q)
    if q.dtype != p.dtype:
        raise ops.BwlaError(2, "gemv_dot needs the GEMV output in the storage type (float64 or float32)")
    return q, ops.dot(p, q, acc=acc)


def gemv_dot_fused(A, p, acc="plain", q=None):
    """q = A p and <p, q> with the inner product in the GEMV's epilogue."""
    return ops.gemv_dot(A, p, acc=acc, out=q)
