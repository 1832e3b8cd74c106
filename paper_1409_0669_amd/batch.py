"""``BatchPlan``: many uneven row-major GEMVs and dots in one batched launch --
one work-group per work item (row tiles of the GEMVs, chunks of the dots,
largest first), one kernel per kind of item (GEMV tiles with x staged in LDS,
the other GEMV tiles, dot chunks), then a finalize kernel that combines each
dot's chunk partials in chunk order -- optionally captured in a HIP graph and
replayed.  The work-group size and the packs of a GEMV row each lane owns come
from the tuning table's batch entry unless given."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from . import ops
from ._lib import BwlaError, check, lib


class BatchPlan:
    """gemvs: list of (A, x, y) with A row-major (contiguous rows, any lda),
    y = A x written in ``out_dtype``.  dots: list of (x, y, out) with out a
    one-element ``out_dtype`` tensor.  All inputs share one storage dtype.
    The plan keeps references to every tensor it was given."""

    def __init__(self, gemvs=(), dots=(), acc="plain", out_dtype=None, grid=0, block=0, packs=0):
        gemvs, dots = list(gemvs), list(dots)
        first = gemvs[0][0] if gemvs else (dots[0][0] if dots else None)
        if first is None:
            raise BwlaError(L.ERR_INVALID_ARG, "empty batch")
        self.dtype, self.device = first.dtype, first.device
        self.out_dtype = ops.default_out_dtype(self.dtype) if out_dtype is None else out_dtype
        self._keep = (gemvs, dots)
        g = (L.GemvDesc * max(1, len(gemvs)))()
        for i, (A, x, y) in enumerate(gemvs):
            layout, lda = ops.matrix_layout(A)
            if layout != L.ROW_MAJOR:
                raise BwlaError(L.ERR_INVALID_ARG, "batched GEMV takes row-major A")
            for t in (A, x):
                if t.dtype != self.dtype or t.device != self.device:
                    raise BwlaError(L.ERR_INVALID_ARG, "gemv %d: dtype/device mismatch" % i)
            if y.dtype != self.out_dtype or y.numel() != A.shape[0] or x.numel() != A.shape[1]:
                raise BwlaError(L.ERR_INVALID_ARG, "gemv %d: x/y shape or y dtype" % i)
            g[i] = L.GemvDesc(A.data_ptr(), A.shape[0], A.shape[1], lda, x.data_ptr(), y.data_ptr())
        d = (L.DotDesc * max(1, len(dots)))()
        for i, (x, y, out) in enumerate(dots):
            if x.dtype != self.dtype or y.dtype != self.dtype or x.numel() != y.numel():
                raise BwlaError(L.ERR_INVALID_ARG, "dot %d: dtype or length mismatch" % i)
            if out.dtype != self.out_dtype or out.numel() != 1:
                raise BwlaError(L.ERR_INVALID_ARG, "dot %d: out must be one %s" % (i, self.out_dtype))
            d[i] = L.DotDesc(x.data_ptr(), y.data_ptr(), x.numel(), out.data_ptr())
        # block (work-group size) and packs (packs of a GEMV row per lane of a
        # staged tile): 0 takes the tuning table's batch entry
        cfg = L.Config(block=int(block), grid=int(grid), unroll=int(packs))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib.bwla_batch_plan_create(ops.dtype_code(self.dtype), ops._ACC[acc],
                                             ops._DTYPE[self.out_dtype], g, len(gemvs), d, len(dots),
                                             ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def info(self):
        items, grid, nbytes = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
        check(lib.bwla_batch_info(self._h, ctypes.byref(items), ctypes.byref(grid), ctypes.byref(nbytes)))
        return {"items": items.value, "grid": grid.value, "bytes": nbytes.value}

    def run(self):
        check(lib.bwla_batch_run(self._h, ops._stream(self.device)))

    def capture(self, stream: torch.cuda.Stream | None = None):
        """Record the plan into a HIP graph on ``stream`` (a created stream,
        default: the current stream).  The capture enqueues nothing."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        check(lib.bwla_batch_capture(self._h, ctypes.c_void_p(s.cuda_stream)))

    def replay(self):
        check(lib.bwla_batch_replay(self._h, ops._stream(self.device)))

    def close(self):
        if getattr(self, "_h", None):
            lib.bwla_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
