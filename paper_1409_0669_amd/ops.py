"""Torch-facing calls of the library: tensors in, tensors out.

PyTorch supplies device memory and the current stream; each function checks
its tensors, then passes raw device pointers, sizes and the stream to the C
ABI, where the HIP kernels do all the work.  Vectors must be contiguous; no
silent copies are made.
"""
from __future__ import annotations

import ctypes
import threading

import torch

from . import _lib as L
from ._lib import BwlaError, check, lib

_DTYPE = {torch.float64: L.F64, torch.float32: L.F32, torch.bfloat16: L.BF16}
_OUT_TORCH = {L.F64: torch.float64, L.F32: torch.float32}
_ACC = {"plain": L.ACC_PLAIN, "compensated": L.ACC_COMPENSATED, L.ACC_PLAIN: L.ACC_PLAIN,
        L.ACC_COMPENSATED: L.ACC_COMPENSATED}


def dtype_code(t: torch.dtype) -> int:
    try:
        return _DTYPE[t]
    except KeyError:
        raise BwlaError(L.ERR_UNSUPPORTED, "dtype %s (supported: float64, float32, bfloat16)" % t)


def compute_dtype(t: torch.dtype) -> torch.dtype:
    """Torch dtype of the compute precision of a storage dtype."""
    return torch.float64 if t == torch.float64 else torch.float32


def default_out_dtype(t: torch.dtype) -> torch.dtype:
    return torch.float64 if t == torch.float64 else torch.float32


# The raw handle of the current stream without building a torch Stream object
# (which costs about 2 us per call, as much as a kernel launch).
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(device=None) -> int:
    """Handle of the current stream of ``device`` (a torch.device or None for
    the current device), as the integer the C ABI takes for ``void *stream``."""
    idx = device.index if device is not None and device.index is not None else None
    if _raw_stream is not None:
        return _raw_stream(torch.cuda.current_device() if idx is None else idx)
    return torch.cuda.current_stream(device).cuda_stream


def _vec(t: torch.Tensor, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise BwlaError(L.ERR_INVALID_ARG, "%s must be a GPU tensor" % name)
    if t.dim() != 1 or not t.is_contiguous():
        raise BwlaError(L.ERR_INVALID_ARG, "%s must be a contiguous 1-D tensor" % name)


def _svec(t: torch.Tensor, name: str) -> int:
    """A 1-D GPU tensor with any positive stride; returns its increment."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise BwlaError(L.ERR_INVALID_ARG, "%s must be a GPU tensor" % name)
    if t.dim() != 1:
        raise BwlaError(L.ERR_INVALID_ARG, "%s must be a 1-D tensor" % name)
    return 1 if t.numel() <= 1 else int(t.stride(0))


def _same(dtype, device, *ts) -> None:
    for t in ts:
        if t.dtype != dtype:
            raise BwlaError(L.ERR_INVALID_ARG, "dtype mismatch: %s vs %s" % (t.dtype, dtype))
        if t.device != device:
            raise BwlaError(L.ERR_INVALID_ARG, "device mismatch: %s vs %s" % (t.device, device))


# ---------------------------------------------------------------------------
# workspace: one buffer per (device, stream), grown on demand
# ---------------------------------------------------------------------------
_ws_lock = threading.Lock()
_ws: dict = {}


def workspace(nbytes: int, device: torch.device, stream: int | None = None) -> torch.Tensor | None:
    """A workspace of at least ``nbytes`` for the current stream (or the
    stream handle given), reused by every call on that stream and reallocated
    only when it must grow.  Grow it before any graph capture with
    :func:`reserve_workspace`."""
    if nbytes == 0:
        return None
    key = (device.index, _stream(device) if stream is None else stream)
    with _ws_lock:
        buf = _ws.get(key)
        if buf is None or buf.numel() < nbytes:
            size = max(nbytes, 1 << 20)
            size = (size + (1 << 20) - 1) >> 20 << 20
            buf = torch.empty(size, dtype=torch.uint8, device=device)
            _ws[key] = buf
        return buf


def reserve_workspace(nbytes: int, device=None) -> None:
    workspace(nbytes, torch.device("cuda", torch.cuda.current_device() if device is None else device))


def _ws_ptr(buf):
    """(address, bytes) of a workspace buffer for the C ABI; (None, 0) for none."""
    return (buf.data_ptr(), buf.numel()) if buf is not None else (None, 0)


# Workspace sizes per (op, dtype, acc, layout, trans, m, n, device): the
# library resolves every pack width and accumulation mode to answer, about as
# long as the launch itself for a small reduction.  The cache is cleared
# whenever the configuration table changes through this module; a table
# changed behind it can only make a call report BWLA_ERR_WORKSPACE, on which
# _with_workspace asks again once.
_ws_sizes: dict = {}


def workspace_size(op: int, dtype: torch.dtype, acc="plain", layout: int = L.ROW_MAJOR, trans: int = 0,
                   m: int = 0, n: int = 0) -> int:
    return _ws_size(torch.cuda.current_device() if torch.cuda.is_initialized() else -1, op, dtype, acc, layout,
                    trans, m, n)


def _ws_size(dev: int, op: int, dtype: torch.dtype, acc, layout: int, trans: int, m: int, n: int) -> int:
    """workspace_size on device index ``dev`` (the current device while the
    library computes the size; -1 before torch has initialised HIP)."""
    key = (op, dtype, acc, layout, trans, m, n, dev)
    v = _ws_sizes.get(key)
    if v is None:
        out = ctypes.c_size_t(0)
        check(lib.bwla_workspace_size(op, dtype_code(dtype), _ACC[acc], layout, trans, m, n, ctypes.byref(out)))
        v = out.value
        if len(_ws_sizes) >= 4096:
            _ws_sizes.clear()
        _ws_sizes[key] = v
    return v


def _with_workspace(size_args, device, stream: int, launch) -> None:
    """Run launch(ws_pointer, ws_bytes) with the stream's workspace at the
    cached size for ``size_args`` (the arguments of :func:`workspace_size`);
    if the library reports the workspace too small, size it afresh and run
    once more (nothing is enqueued by a call that fails validation).  The
    tensors are on ``device``, which the caller's stream belongs to; the
    sizes are cached under its index."""
    if device is not None and device.index is not None:
        dev = device.index
    else:
        dev = torch.cuda.current_device() if torch.cuda.is_initialized() else -1
    st = launch(*_ws_ptr(workspace(_ws_size(dev, *size_args), device, stream)))
    if st == L.ERR_WORKSPACE:
        _ws_sizes.clear()
        st = launch(*_ws_ptr(workspace(_ws_size(dev, *size_args), device, stream)))
    check(st)


# ---------------------------------------------------------------------------
# operations
# ---------------------------------------------------------------------------
def copy(y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """x <- y.  Strided 1-D views are accepted (increment = stride)."""
    incy = _svec(y, "y")
    x = torch.empty(y.numel(), dtype=y.dtype, device=y.device) if out is None else out
    incx = _svec(x, "out")
    _same(y.dtype, y.device, x)
    if x.numel() != y.numel():
        raise BwlaError(L.ERR_INVALID_ARG, "length mismatch")
    if incx == 1 and incy == 1:
        check(lib.bwla_copy(dtype_code(y.dtype), y.numel(), y.data_ptr(), x.data_ptr(), _stream(y.device)))
    else:
        check(lib.bwla_copy_strided(dtype_code(y.dtype), y.numel(), y.data_ptr(), incy, x.data_ptr(), incx,
                                    _stream(y.device)))
    return x


def axpby(alpha: float, y: torch.Tensor, beta: float, z: torch.Tensor, out: torch.Tensor | None = None,
          alpha_dev: torch.Tensor | None = None, beta_dev: torch.Tensor | None = None) -> torch.Tensor:
    """x <- alpha*y + beta*z, computed as RN(fma(a, y, RN(b*z))) in the compute
    precision.  ``out`` may be ``y`` or ``z`` (in-place).  ``alpha_dev`` /
    ``beta_dev``: optional one-element device tensors of the compute dtype that
    multiply the host factors.  Strided 1-D views are accepted."""
    incy = _svec(y, "y")
    incz = _svec(z, "z")
    _same(y.dtype, y.device, z)
    x = torch.empty(y.numel(), dtype=y.dtype, device=y.device) if out is None else out
    incx = _svec(x, "out")
    _same(y.dtype, y.device, x)
    if not (x.numel() == y.numel() == z.numel()):
        raise BwlaError(L.ERR_INVALID_ARG, "length mismatch")
    ad, bd = _dev_scalar(y, alpha_dev, "alpha_dev"), _dev_scalar(y, beta_dev, "beta_dev")
    if incx == incy == incz == 1:
        check(lib.bwla_axpby(dtype_code(y.dtype), y.numel(), float(alpha), ad, y.data_ptr(), float(beta), bd,
                             z.data_ptr(), x.data_ptr(), _stream(y.device)))
    else:
        check(lib.bwla_axpby_strided(dtype_code(y.dtype), y.numel(), float(alpha), ad, y.data_ptr(), incy,
                                     float(beta), bd, z.data_ptr(), incz, x.data_ptr(), incx, _stream(y.device)))
    return x


def _dev_scalar(like: torch.Tensor, s: torch.Tensor | None, name: str):
    if s is None:
        return None
    cd = compute_dtype(like.dtype)
    if s.dtype != cd or s.numel() != 1 or s.device != like.device:
        raise BwlaError(L.ERR_INVALID_ARG, "%s must be one %s element on %s" % (name, cd, like.device))
    return s.data_ptr()


def scal(alpha: float, x: torch.Tensor, alpha_dev: torch.Tensor | None = None) -> torch.Tensor:
    """x <- alpha x in place (x_i = RN(a x_i)); strided 1-D views accepted."""
    incx = _svec(x, "x")
    check(lib.bwla_scal(dtype_code(x.dtype), x.numel(), float(alpha), _dev_scalar(x, alpha_dev, "alpha_dev"),
                        x.data_ptr(), incx, _stream(x.device)))
    return x


def scal_to(alpha: float, y: torch.Tensor, out: torch.Tensor | None = None,
            alpha_dev: torch.Tensor | None = None) -> torch.Tensor:
    """x <- alpha y out of place (x_i = RN(a y_i), one product per element);
    contiguous 1-D tensors.  ``alpha_dev``: an optional one-element device
    tensor of the compute dtype that multiplies alpha (the upstream gradient
    of an inner product, left on the device)."""
    _vec(y, "y")
    x = torch.empty_like(y) if out is None else out
    _vec(x, "out")
    _same(y.dtype, y.device, x)
    if x.numel() != y.numel():
        raise BwlaError(L.ERR_INVALID_ARG, "length mismatch")
    check(lib.bwla_scal_to(dtype_code(y.dtype), y.numel(), float(alpha), _dev_scalar(y, alpha_dev, "alpha_dev"),
                           y.data_ptr(), x.data_ptr(), _stream(y.device)))
    return x


def _scalar_out(dtype, out_dtype, device, out):
    od = default_out_dtype(dtype) if out_dtype is None else out_dtype
    if od not in (torch.float64, torch.float32):
        raise BwlaError(L.ERR_UNSUPPORTED, "output dtype %s" % od)
    if out is None:
        out = torch.empty((), dtype=od, device=device)
    elif out.dtype != od or out.numel() != 1 or out.device != device:
        raise BwlaError(L.ERR_INVALID_ARG, "out must be one %s element on %s" % (od, device))
    return out, _DTYPE[od]


def dot(x: torch.Tensor, y: torch.Tensor, acc="plain", out_dtype: torch.dtype | None = None,
        out: torch.Tensor | None = None) -> torch.Tensor:
    """<x, y> as a 0-dim device tensor (float64 for f64 input, float32 by
    default otherwise).  Strided 1-D views are accepted."""
    incx = _svec(x, "x")
    incy = _svec(y, "y")
    _same(x.dtype, x.device, y)
    if x.numel() != y.numel():
        raise BwlaError(L.ERR_INVALID_ARG, "length mismatch")
    out, oc = _scalar_out(x.dtype, out_dtype, x.device, out)
    args = (dtype_code(x.dtype), _ACC[acc], x.numel(), x.data_ptr(), incx, y.data_ptr(), incy, oc, out.data_ptr())
    stream = _stream(x.device)
    _with_workspace((L.OP_DOT, x.dtype, acc, L.ROW_MAJOR, 0, 0, x.numel()), x.device, stream,
                    lambda ws, wsn: lib.bwla_dot_strided(*args, ws, wsn, stream))
    return out


def dot_noalloc(x: torch.Tensor, y: torch.Tensor, acc="plain", out_dtype: torch.dtype | None = None,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """<x, y> as :func:`dot` computes it (bitwise the same), with the
    partials in the library's static device scratch instead of a workspace:
    nothing is allocated when ``out`` is given.  Contiguous 1-D tensors.
    Calls that may overlap on one GPU race on that scratch."""
    _vec(x, "x")
    _vec(y, "y")
    _same(x.dtype, x.device, y)
    if x.numel() != y.numel():
        raise BwlaError(L.ERR_INVALID_ARG, "length mismatch")
    out, oc = _scalar_out(x.dtype, out_dtype, x.device, out)
    check(lib.bwla_dot_noalloc(dtype_code(x.dtype), _ACC[acc], x.numel(), x.data_ptr(), y.data_ptr(), oc,
                               out.data_ptr(), _stream(x.device)))
    return out


def nrm2(x: torch.Tensor, acc="plain", out_dtype: torch.dtype | None = None,
         out: torch.Tensor | None = None) -> torch.Tensor:
    """sqrt(<x, x>) as a 0-dim device tensor; strided 1-D views accepted."""
    incx = _svec(x, "x")
    out, oc = _scalar_out(x.dtype, out_dtype, x.device, out)
    args = (dtype_code(x.dtype), _ACC[acc], x.numel(), x.data_ptr(), incx, oc, out.data_ptr())
    stream = _stream(x.device)
    _with_workspace((L.OP_DOT, x.dtype, acc, L.ROW_MAJOR, 0, 0, x.numel()), x.device, stream,
                    lambda ws, wsn: lib.bwla_nrm2_strided(*args, ws, wsn, stream))
    return out


def asum(x: torch.Tensor, acc="plain", out_dtype: torch.dtype | None = None,
         out: torch.Tensor | None = None) -> torch.Tensor:
    """sum |x_i| as a 0-dim device tensor; strided 1-D views accepted."""
    incx = _svec(x, "x")
    out, oc = _scalar_out(x.dtype, out_dtype, x.device, out)
    args = (dtype_code(x.dtype), _ACC[acc], x.numel(), x.data_ptr(), incx, oc, out.data_ptr())
    stream = _stream(x.device)
    _with_workspace((L.OP_DOT, x.dtype, acc, L.ROW_MAJOR, 0, 0, x.numel()), x.device, stream,
                    lambda ws, wsn: lib.bwla_asum(*args, ws, wsn, stream))
    return out


def matrix_layout(A: torch.Tensor):
    """(layout, lda) of a 2-D tensor whose rows or columns are contiguous."""
    if A.dim() != 2:
        raise BwlaError(L.ERR_INVALID_ARG, "A must be 2-D")
    m, n = A.shape
    s0, s1 = A.stride()
    if s1 == 1 and (s0 >= max(1, n) or m <= 1):
        return L.ROW_MAJOR, max(s0, n, 1)
    if s0 == 1 and (s1 >= max(1, m) or n <= 1):
        return L.COL_MAJOR, max(s1, m, 1)
    raise BwlaError(L.ERR_INVALID_ARG, "A must have contiguous rows or columns (strides %s)" % (A.stride(),))


def gemv(A: torch.Tensor, x: torch.Tensor, trans: bool = False, acc="plain",
         out_dtype: torch.dtype | None = None, out: torch.Tensor | None = None, alpha: float = 1.0,
         beta: float = 0.0) -> torch.Tensor:
    """y = alpha op(A) x + beta y with op(A) = A or A^T (alpha = 1, beta = 0:
    y = op(A) x, y not read).  The layout (row- or column-major, with leading
    dimension) is read from A's strides; x and ``out`` may be strided 1-D
    views.  beta != 0 needs ``out`` (it is read)."""
    if not A.is_cuda:
        raise BwlaError(L.ERR_INVALID_ARG, "A must be a GPU tensor")
    layout, lda = matrix_layout(A)
    incx = _svec(x, "x")
    _same(A.dtype, A.device, x)
    m, n = A.shape
    out_len, in_len = (n, m) if trans else (m, n)
    if x.numel() != in_len:
        raise BwlaError(L.ERR_INVALID_ARG, "x has %d entries, op(A) has %d columns" % (x.numel(), in_len))
    od = default_out_dtype(A.dtype) if out_dtype is None else out_dtype
    if od not in (torch.float64, torch.float32):
        raise BwlaError(L.ERR_UNSUPPORTED, "output dtype %s" % od)
    if beta != 0.0 and out is None:
        raise BwlaError(L.ERR_INVALID_ARG, "beta != 0 needs out (y is read)")
    y = torch.empty(out_len, dtype=od, device=A.device) if out is None else out
    incy = _svec(y, "out")
    if y.numel() != out_len or y.dtype != od:
        raise BwlaError(L.ERR_INVALID_ARG, "out must have %d %s entries" % (out_len, od))
    if alpha == 1.0 and beta == 0.0 and incx == 1 and incy == 1:
        args = (dtype_code(A.dtype), _ACC[acc], layout, int(trans), m, n, A.data_ptr(), lda, x.data_ptr(),
                _DTYPE[od], y.data_ptr())
        stream = _stream(A.device)
        _with_workspace((L.OP_GEMV_ROWS, A.dtype, acc, layout, int(trans), m, n), A.device, stream,
                        lambda ws, wsn: lib.bwla_gemv(*args, ws, wsn, stream))
        return y
    nbytes = ctypes.c_size_t()
    check(lib.bwla_gemv_ex_workspace_size(dtype_code(A.dtype), _DTYPE[od], layout, int(trans), m, n,
                                          ctypes.byref(nbytes)))
    ws, wsn = _ws_ptr(workspace(nbytes.value, A.device))
    check(lib.bwla_gemv_ex(dtype_code(A.dtype), _ACC[acc], layout, int(trans), m, n, float(alpha), A.data_ptr(),
                           lda, x.data_ptr(), incx, float(beta), _DTYPE[od], y.data_ptr(), incy, ws, wsn,
                           _stream(A.device)))
    return y


def gemv_dot(A: torch.Tensor, x: torch.Tensor, w: torch.Tensor | None = None, trans: bool = False,
             acc="plain", dot_dtype: torch.dtype | None = None, out: torch.Tensor | None = None,
             dot_out: torch.Tensor | None = None):
    """(y, s): y = op(A) x in A's dtype (float64 or float32) and s = <w, y> in
    one fused launch sequence.  ``w`` defaults to ``x`` (the q = A p, <p, q>
    pair of a conjugate-gradient iteration; op(A) must then be square)."""
    if not A.is_cuda:
        raise BwlaError(L.ERR_INVALID_ARG, "A must be a GPU tensor")
    if A.dtype not in (torch.float64, torch.float32):
        raise BwlaError(L.ERR_UNSUPPORTED, "gemv_dot stores y in A's dtype: float64 or float32")
    layout, lda = matrix_layout(A)
    w = x if w is None else w
    _vec(x, "x")
    _vec(w, "w")
    _same(A.dtype, A.device, x, w)
    m, n = A.shape
    out_len, in_len = (n, m) if trans else (m, n)
    if x.numel() != in_len or w.numel() != out_len:
        raise BwlaError(L.ERR_INVALID_ARG, "x needs %d entries and w %d" % (in_len, out_len))
    y = torch.empty(out_len, dtype=A.dtype, device=A.device) if out is None else out
    _vec(y, "out")
    if y.numel() != out_len or y.dtype != A.dtype:
        raise BwlaError(L.ERR_INVALID_ARG, "out must have %d %s entries" % (out_len, A.dtype))
    s, sc = _scalar_out(A.dtype, dot_dtype, A.device, dot_out)
    nbytes = ctypes.c_size_t()
    check(lib.bwla_gemv_dot_workspace_size(dtype_code(A.dtype), layout, int(trans), m, n, ctypes.byref(nbytes)))
    ws, wsn = _ws_ptr(workspace(nbytes.value, A.device))
    check(lib.bwla_gemv_dot(dtype_code(A.dtype), _ACC[acc], layout, int(trans), m, n, A.data_ptr(), lda,
                            x.data_ptr(), y.data_ptr(), w.data_ptr(), sc, s.data_ptr(), ws, wsn,
                            _stream(A.device)))
    return y, s


def ger(u: torch.Tensor, v: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """A <- u v^T (overwrite), every entry rounded once to A's dtype.  ``out``
    is the m x n matrix to overwrite; its layout is read from its strides."""
    _vec(u, "u")
    _vec(v, "v")
    _same(out.dtype, out.device, u, v)
    layout, lda = matrix_layout(out)
    m, n = out.shape
    if u.numel() != m or v.numel() != n:
        raise BwlaError(L.ERR_INVALID_ARG, "u, v must have %d and %d entries" % (m, n))
    check(lib.bwla_ger(dtype_code(out.dtype), layout, m, n, u.data_ptr(), v.data_ptr(), out.data_ptr(), lda,
                       _stream(out.device)))
    return out


def cg_update(alpha: float, x: torch.Tensor, p: torch.Tensor, r: torch.Tensor, q: torch.Tensor, acc="plain",
              out_dtype: torch.dtype | None = None, alpha_dev: torch.Tensor | None = None,
              out: torch.Tensor | None = None) -> torch.Tensor:
    """One fused pass: x += a p, r -= a q, returns <r, r> (0-dim tensor)."""
    for name, t in (("x", x), ("p", p), ("r", r), ("q", q)):
        _vec(t, name)
    _same(x.dtype, x.device, p, r, q)
    if not (x.numel() == p.numel() == r.numel() == q.numel()):
        raise BwlaError(L.ERR_INVALID_ARG, "length mismatch")
    if alpha_dev is not None and (alpha_dev.dtype != compute_dtype(x.dtype) or alpha_dev.numel() != 1):
        raise BwlaError(L.ERR_INVALID_ARG, "alpha_dev must be one %s element" % compute_dtype(x.dtype))
    out, oc = _scalar_out(x.dtype, out_dtype, x.device, out)
    args = (dtype_code(x.dtype), _ACC[acc], x.numel(), float(alpha), None if alpha_dev is None else alpha_dev.data_ptr(),
            x.data_ptr(), p.data_ptr(), r.data_ptr(), q.data_ptr(), oc, out.data_ptr())
    stream = _stream(x.device)
    _with_workspace((L.OP_DOT, x.dtype, acc, L.ROW_MAJOR, 0, 0, x.numel()), x.device, stream,
                    lambda ws, wsn: lib.bwla_cg_update(*args, ws, wsn, stream))
    return out


# ---------------------------------------------------------------------------
# configuration
# ---------------------------------------------------------------------------
def set_config(op: int, dtype: torch.dtype, size_class: int = -1, acc=None, **fields) -> None:
    """Set the configuration of (op, dtype, accumulation mode, size class); no
    fields = defaults.  acc None sets both accumulation modes."""
    a = -1 if acc is None else _ACC[acc]
    _ws_sizes.clear()
    if fields:
        c = L.Config(**{k: int(v) for k, v in fields.items()})
        check(lib.bwla_set_config(op, dtype_code(dtype), a, size_class, ctypes.byref(c)))
    else:
        check(lib.bwla_set_config(op, dtype_code(dtype), a, size_class, None))


def get_config(op: int, dtype: torch.dtype, m: int = 0, n: int = 0, acc="plain") -> dict:
    c = L.Config()
    check(lib.bwla_get_config(op, dtype_code(dtype), _ACC[acc], m, n, ctypes.byref(c)))
    return c.as_dict()


def load_tuning(path: str) -> None:
    _ws_sizes.clear()
    check(lib.bwla_load_tuning(path.encode()))


def default_table_path() -> str:
    import os
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "gfx950.txt")


def load_default_tuning() -> bool:
    """Load the tuning table shipped with the package (measured on MI355X),
    unless BWLA_TUNING names another table (the library loads that one itself).
    Returns True if the shipped table was loaded."""
    import os
    if os.environ.get("BWLA_TUNING"):
        return False
    path = default_table_path()
    if os.path.exists(path):
        load_tuning(path)
        return True
    return False


def reset_config() -> None:
    for op in range(L.OP_COUNT):
        for t in (torch.float64, torch.float32, torch.bfloat16):
            set_config(op, t)


load_default_tuning()
