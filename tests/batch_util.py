"""Uneven problem sets for the batched-launch tests (test helper)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import workloads as W
from tests.criteria import TOL, check_scalar, check_vector, cond_scale, plain_reduced
from tests.gpu_util import guarded, host


def problems(dtype, n_gemv, n_dot, gemv_hi, dot_hi, seed=0, align=64):
    """Device buffers sliced into uneven problems (starts aligned to `align`
    elements) and the host float64 copies."""
    rng = np.random.default_rng(seed)
    Ms = rng.integers(1, gemv_hi + 1, n_gemv)
    Ns = rng.integers(1, gemv_hi + 1, n_gemv)
    Ds = rng.integers(0, dot_hi + 1, n_dot)
    return from_sizes(dtype, Ms, Ns, Ds, seed, align)


def from_sizes(dtype, Ms, Ns, Ds, seed=0, align=64, guards=None, od=None):
    """As problems(), from given sizes.  With a list ``guards``, every output
    sits between sentinel slack (tests.gpu_util.guarded) and the list
    receives each output's check.  ``od``: the output dtype (default float64
    for f64 storage, else float32)."""
    def off(sizes):
        o, offs = 0, []
        for s in sizes:
            offs.append(o)
            o += (int(s) + align - 1) // align * align
        return offs, max(o, 1)
    a_off, a_tot = off(Ms * Ns)
    x_off, x_tot = off(Ns)
    d_off, d_tot = off(Ds)
    A = W.device_draw(a_tot, dtype, seed, 501)
    X = W.device_draw(x_tot, dtype, seed, 502)
    P = W.device_draw(d_tot, dtype, seed, 503)
    Q = W.device_draw(d_tot, dtype, seed, 504)
    if od is None:
        od = torch.float64 if dtype == "f64" else torch.float32
    gemvs = []
    for i, (m, n) in enumerate(zip(Ms, Ns)):
        m, n = int(m), int(n)
        Ai = A[a_off[i]:a_off[i] + m * n].view(m, n)
        xi = X[x_off[i]:x_off[i] + n]
        gemvs.append((Ai, xi, _out(m, od, guards, "gemv %d" % i)))
    dots = []
    for i, n in enumerate(Ds):
        n = int(n)
        dots.append((P[d_off[i]:d_off[i] + n], Q[d_off[i]:d_off[i] + n], _out(1, od, guards, "dot %d" % i)))
    return gemvs, dots


def _out(n, od, guards, what):
    if guards is None:
        return torch.empty(n, dtype=od, device="cuda")
    view, check = guarded(n, od)
    guards.append(lambda: check(what))
    return view


def check(dtype, acc, gemvs, dots, gi=None, di=None):
    """Every problem (or those indexed by gi, di) against the oracle under
    the criteria of tests/criteria.py for storage ``dtype`` and accumulation
    ``acc``."""
    gi = range(len(gemvs)) if gi is None else gi
    di = range(len(dots)) if di is None else di
    for i in gi:
        A, x, y = gemvs[i]
        A64, x64 = host(A), host(x)
        ref = oracle.gemv(A64, x64)
        check_vector(host(y), ref, np.abs(A64) @ np.abs(x64), TOL[dtype], "gemv %d" % i,
                     plain_f32=plain_reduced(dtype, acc))
    for i in di:
        p, q, out = dots[i]
        p64, q64 = host(p), host(q)
        check_scalar(float(out.item()), oracle.dot(p64, q64), cond_scale(dtype, acc, np.abs(p64 * q64).sum()),
                     TOL[dtype], "dot %d" % i)


