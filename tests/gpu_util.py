"""Shared helpers of the GPU parity tests (test helper)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import workloads as W

DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
PREC = {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16"}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def vec(n, dtype, stream, seed=0, dist="uniform", pad_front=0):
    """(device tensor, exact float64 values).  pad_front > 0 places the vector
    that many elements into a larger buffer, so its address is misaligned."""
    s, x = W.vector(n, dtype, seed=seed, stream=stream, dist=dist)
    t = W.to_torch(s, dtype)
    if pad_front:
        buf = torch.zeros(n + pad_front, dtype=DT[dtype], device="cuda")
        buf[pad_front:] = t
        t = buf[pad_front:]
    return t, x


def mat(m, n, dtype, stream, layout="row", seed=0, dist="uniform", pad=0):
    """(device m x n tensor in the given layout with leading dimension padded
    by `pad`, exact float64 m x n array)."""
    s, a = W.vector(m * n, dtype, seed=seed, stream=stream, dist=dist)
    a = a.reshape(m, n)
    s = s.reshape(m, n)
    if layout == "row":
        buf = np.zeros((m, n + pad), dtype=s.dtype)
        buf[:, :n] = s
        t = W.to_torch(buf, dtype)[:, :n]
    else:
        buf = np.zeros((n, m + pad), dtype=s.dtype)
        buf[:, :m] = s.T
        t = W.to_torch(buf, dtype)[:, :m].t()
    return t, a


def host(t, dtype=None):
    dtype = dtype or PREC[t.dtype]
    return W.from_torch(t, dtype)


# Guard slack around outputs: the output lives inside a larger buffer whose
# GUARD_BYTES before and after hold a NaN bit pattern no kernel computes; the
# test checks after the call that every slack entry still holds it, which
# catches stores past either end of the output (tail handling, split slices).
GUARD_BYTES = 4096
_SENTINEL = {torch.float64: (torch.int64, 0x7FF4DEADBEEF0001), torch.float32: (torch.int32, 0x7FA0DEAD),
             torch.bfloat16: (torch.int16, 0x7FA5)}


def guarded(n, dtype, offset=0):
    """(view, check): an output of n entries of ``dtype`` (torch dtype or a
    short name), ``offset`` entries past an aligned start, with sentinel
    slack on both sides; check() asserts the slack is untouched."""
    dt = DT.get(dtype, dtype)
    it, bits = _SENTINEL[dt]
    g = GUARD_BYTES // torch.empty(0, dtype=dt).element_size()
    buf = torch.full((n + offset + 2 * g,), bits, dtype=it, device="cuda")
    view = buf.view(dt)[g + offset:g + offset + n]
    if n == 0:
        view = view.reshape(0)

    def check(what=""):
        h = buf.cpu()
        lo = int((h[:g + offset] != bits).sum())
        hi = int((h[g + offset + n:] != bits).sum())
        assert lo == 0 and hi == 0, "%s: %d guard entries before and %d after the output were written" % (
            what, lo, hi)
    return view, check


def guarded_scalar(dtype):
    """A 0-dim guarded output (for the reductions)."""
    v, check = guarded(1, dtype)
    return v.view(()), check
