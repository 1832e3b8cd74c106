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
