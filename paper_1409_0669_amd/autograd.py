"""Autograd functions with hand-written backward kernels.

* ``GemvFn``: y = A x.  Backward: dx = A^T ybar (the transposed-layout GEMV
  kernel on the same bytes of A) and dA = ybar x^T (the rank-1 overwrite
  kernel, a bandwidth-bound write of A's size), each only when needed.
* ``DotFn``: z = <x, y>.  Backward: dx = RN(zbar * y) and dy = RN(zbar * x),
  each one out-of-place scaling (one product per element, one read and one
  write) whose factor zbar stays on the device.

Storage types float64 and float32 (GEMV); float64, float32 and bfloat16 (dot).
Results and gradients of reductions are in the compute precision.
"""
from __future__ import annotations

import torch

from . import ops


class GemvFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A: torch.Tensor, x: torch.Tensor, acc="plain"):
        if A.dtype not in (torch.float64, torch.float32):
            raise ops.BwlaError(2, "GemvFn supports float64 and float32 storage")
        y = ops.gemv(A, x, acc=acc, out_dtype=A.dtype)
        ctx.save_for_backward(A, x)
        ctx.acc = acc
        return y

    @staticmethod
    def backward(ctx, ybar: torch.Tensor):
        A, x = ctx.saved_tensors
        ybar = ybar.contiguous()
        dA = dx = None
        if ctx.needs_input_grad[1]:
            dx = ops.gemv(A, ybar, trans=True, acc=ctx.acc, out_dtype=A.dtype)
        if ctx.needs_input_grad[0]:
            dA = torch.empty_strided(A.shape, A.stride(), dtype=A.dtype, device=A.device)
            ops.ger(ybar, x.contiguous(), dA)  # the rank-1 kernel reads unit-stride vectors
        return dA, dx, None


class DotFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, y: torch.Tensor, acc="plain"):
        z = ops.dot(x, y, acc=acc, out_dtype=ops.compute_dtype(x.dtype))
        ctx.save_for_backward(x, y)
        return z

    @staticmethod
    def backward(ctx, zbar: torch.Tensor):
        x, y = ctx.saved_tensors
        zb = zbar.reshape(1).contiguous()
        dx = dy = None
        if ctx.needs_input_grad[0]:
            dx = ops.scal_to(1.0, y, alpha_dev=zb)
        if ctx.needs_input_grad[1]:
            dy = ops.scal_to(1.0, x, alpha_dev=zb)
        return dx, dy, None


def gemv(A, x, acc="plain"):
    return GemvFn.apply(A, x, acc)


def dot(x, y, acc="plain"):
    return DotFn.apply(x, y, acc)
