"""Seeded synthetic inputs for the bandwidth-limited BLAS-1/2 workloads.

This module only draws random numbers and converts them to storage formats; it
holds none of the operations' arithmetic.  Both the CPU oracle's tests and the
GPU path's tests and benchmark draw their inputs from here, so the two sides see
the same stored values.

Recipe (used everywhere):

* Every tensor has its own stream: ``numpy.random.default_rng(SeedSequence([seed, k]))``
  for a caller-chosen tensor index ``k``, so draws do not depend on the order in
  which tensors are generated.
* Values are drawn in float64: uniform on [-1, 1) or standard normal.  The paper
  states no value distribution; these are the distributions of the workloads.
* Storage conversion rounds to nearest-even: float64 -> float32 (numpy), and
  float32 -> bfloat16 (torch's CPU conversion).  Widening back to float64 is exact.
* Problem sizes of the batched workload are ``round(exp(U(ln lo, ln hi)))``,
  clamped to [lo, hi].
"""
from __future__ import annotations

import numpy as np

DTYPES = ("f64", "f32", "bf16")
ITEMSIZE = {"f64": 8, "f32": 4, "bf16": 2}


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


def uniform(n, seed: int = 0, stream: int = 0) -> np.ndarray:
    """float64 draws on [-1, 1)."""
    return rng(seed, stream).uniform(-1.0, 1.0, size=n)


def normal(n, seed: int = 0, stream: int = 0) -> np.ndarray:
    """float64 standard-normal draws."""
    return rng(seed, stream).standard_normal(size=n)


def draw(dist: str, n, seed: int = 0, stream: int = 0) -> np.ndarray:
    if dist == "uniform":
        return uniform(n, seed, stream)
    if dist == "normal":
        return normal(n, seed, stream)
    raise ValueError(dist)


def quantize(a: np.ndarray, dtype: str) -> np.ndarray:
    """Round float64 values to the storage format.  bf16 is returned as uint16
    bit patterns."""
    a = np.asarray(a, dtype=np.float64)
    if dtype == "f64":
        return a.copy()
    f32 = a.astype(np.float32)
    if dtype == "f32":
        return f32
    if dtype == "bf16":
        import torch
        t = torch.from_numpy(np.ascontiguousarray(f32)).to(torch.bfloat16)
        return t.view(torch.int16).numpy().view(np.uint16).copy()
    raise ValueError(dtype)


def widen(stored: np.ndarray, dtype: str) -> np.ndarray:
    """Exact float64 values of stored elements."""
    if dtype == "bf16":
        bits = stored.astype(np.uint32) << np.uint32(16)
        return bits.view(np.float32).astype(np.float64)
    return np.asarray(stored).astype(np.float64)


def to_torch(stored: np.ndarray, dtype: str, device="cuda"):
    """Upload stored values as a torch tensor of the storage dtype."""
    import torch
    if dtype == "bf16":
        t = torch.from_numpy(np.ascontiguousarray(stored).view(np.int16)).view(torch.bfloat16)
    else:
        t = torch.from_numpy(np.ascontiguousarray(stored))
    return t.to(device)


def from_torch(t, dtype: str) -> np.ndarray:
    """Download a tensor and return the exact float64 values of its elements."""
    import torch
    t = t.detach().to("cpu").contiguous()
    if dtype == "bf16":
        return widen(t.view(torch.int16).numpy().view(np.uint16), "bf16")
    return t.numpy().astype(np.float64)


def vector(n: int, dtype: str, seed: int = 0, stream: int = 0, dist: str = "uniform"):
    """(stored, exact float64) pair for a length-n vector."""
    s = quantize(draw(dist, n, seed, stream), dtype)
    return s, widen(s, dtype)


def device_draw(n, dtype: str, seed: int = 0, stream: int = 0, dist: str = "uniform", device="cuda"):
    """Seeded draws generated directly in device memory (for inputs too large
    to draw on the host quickly): torch's Philox generator on the device,
    seeded from SeedSequence([seed, stream]); float64 uniform on [-1, 1) or
    standard normal, rounded to the storage type (f64 -> f32 -> bf16, nearest
    even).  Download with :func:`from_torch` for exact float64 values."""
    import torch
    state = int(np.random.SeedSequence([int(seed), int(stream)]).generate_state(1, np.uint64)[0])
    g = torch.Generator(device=device)
    g.manual_seed(state & ((1 << 63) - 1))
    if dist == "uniform":
        t = torch.rand(n, generator=g, dtype=torch.float64, device=device).mul_(2.0).sub_(1.0)
    elif dist == "normal":
        t = torch.randn(n, generator=g, dtype=torch.float64, device=device)
    else:
        raise ValueError(dist)
    if dtype == "f64":
        return t
    t = t.to(torch.float32)
    return t if dtype == "f32" else t.to(torch.bfloat16)


def loguniform_sizes(lo: int, hi: int, count: int, seed: int = 0, stream: int = 0) -> np.ndarray:
    u = rng(seed, stream).uniform(np.log(lo), np.log(hi), size=count)
    return np.clip(np.rint(np.exp(u)), lo, hi).astype(np.int64)


# ---------------------------------------------------------------------------
# Workload shapes.  Names describe the workloads; sizes follow the paper's
# experiments scaled to a 288 GB HBM3E device.
# ---------------------------------------------------------------------------

#: small FP64 set: vectors of 2^20 entries and a 1024 x 1024 row-major matrix.
SMALL_FP64 = {"n": 1 << 20, "gemv": (1024, 1024), "dtype": "f64", "dist": "uniform"}

#: plain kernels at paper scale.
PAPER_SCALE = {
    "vector_sizes": (10 ** 5, 10 ** 6, 10 ** 7, 1 << 26),
    "gemv_shapes": ((4096, 4096), (16384, 16384)),
    "dtypes": ("f32", "f64"),
    "layouts": ("row", "col"),
    "dist": "uniform",
}

#: composite CG-like step and GEMV followed by a dot.
COMPOSITE = {"n": 1 << 24, "gemv": (8192, 8192), "dtype": "f64", "dist": "normal"}

#: differentiation shapes.
ADJOINT = {"gemv_shapes": ((4096, 4096), (16384, 2048), (2048, 16384)), "dot_n": 1 << 24,
           "dtype": "f32", "fd_shapes": ((64, 48), (8, 8))}

#: batched uneven workload.
BATCHED = {"n_gemv": 512, "gemv_lo": 32, "gemv_hi": 4096, "n_dot": 4096,
           "dot_lo": 10 ** 3, "dot_hi": 10 ** 6, "dtypes": ("bf16", "f32")}


def batched_sizes(seed: int = 0, n_gemv: int = 512, n_dot: int = 4096,
                  gemv_lo: int = 32, gemv_hi: int = 4096, dot_lo: int = 10 ** 3,
                  dot_hi: int = 10 ** 6):
    """Sizes of the batched workload: (M[], N[]) for the GEMVs and n[] for the dots."""
    M = loguniform_sizes(gemv_lo, gemv_hi, n_gemv, seed, 1001)
    N = loguniform_sizes(gemv_lo, gemv_hi, n_gemv, seed, 1002)
    D = loguniform_sizes(dot_lo, dot_hi, n_dot, seed, 1003)
    return M, N, D
