"""CPU oracle for the bandwidth-limited BLAS-1/2 operations of Rupp et al.,
"Performance Portability Study of Linear Algebra Kernels in OpenCL" (IWOCL 2014).

TEST INFRASTRUCTURE ONLY.  The functions here are the parity reference that the
GPU library is checked against.  They share no code with the GPU path and the
GPU path never imports them; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.

Every function takes numpy float64 arrays holding the exact stored values of
the operands (f32 and bf16 operands widened exactly) and returns float64
arrays.  The arithmetic lives in ``oracle.c`` (plain C, double precision,
compiled with ``-ffp-contract=off``); this module only marshals arguments.
Operation definitions follow Section 2 of the paper:

* ``copy``   x <- y
* ``axpby``  x <- alpha*y + beta*z        (rounding sequence RN(alpha*y + RN(beta*z)))
* ``dot``    <x, y>                       (Dot2 compensated evaluation)
* ``nrm2``   sqrt(<x, x>)
* ``gemv``   y <- op(A) x, row- or column-major A
* ``ger``    A <- u v^T                   (gradient of y = A x with respect to A)
* ``gemv_dot`` y <- op(A) x stored in the storage precision, then <w, y>: the
  GEMV-then-inner-product pair of a conjugate-gradient iteration, a composite
  of the two definitions above
* ``scal``   x <- alpha*y, one rounding    (BLAS scal)
* ``asum``   sum |x_i|                     (BLAS asum, Sum2 compensated evaluation)
* ``strided`` / ``scatter``  the BLAS increment convention for vectors
* ``gemv_axpby``  y <- alpha op(A) x + beta y as the composite of ``gemv``,
  rounding to the output precision, and ``axpby`` (``scal`` when beta == 0,
  so that y is not read)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

F64, F32, BF16 = 0, 1, 2
ROW_MAJOR, COL_MAJOR = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# ORACLE_LIBRARY may name another build of oracle.c (the sanitizer build of
# build_sanitized()); by default the in-tree one is loaded.
_LOAD = os.environ.get("ORACLE_LIBRARY") or _LIB

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (no GPU code)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out_path: str) -> str:
    """Compile ``oracle.c`` with gcc's AddressSanitizer and
    UndefinedBehaviorSanitizer (any finding ends the process) into
    ``out_path``; a process loads it with gcc's libasan preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", out_path, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LOAD == _LIB and not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LOAD)
    dp = ctypes.POINTER(ctypes.c_double)
    i64, c_int, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.o_round_bf16.argtypes = [dbl]
    lib.o_round_bf16.restype = dbl
    lib.o_scalar.argtypes = [c_int, dbl, c_int, dbl]
    lib.o_scalar.restype = dbl
    lib.o_copy.argtypes = [i64, dp, dp]
    lib.o_copy.restype = None
    lib.o_axpby.argtypes = [c_int, i64, dbl, dp, dbl, dp, dp]
    lib.o_axpby.restype = None
    lib.o_dot.argtypes = [i64, dp, i64, dp, i64]
    lib.o_dot.restype = dbl
    lib.o_nrm2.argtypes = [i64, dp]
    lib.o_nrm2.restype = dbl
    lib.o_gemv.argtypes = [c_int, c_int, i64, i64, dp, i64, dp, dp]
    lib.o_gemv.restype = None
    lib.o_ger.argtypes = [c_int, c_int, i64, i64, dp, dp, dp, i64]
    lib.o_ger.restype = None
    lib.o_scal.argtypes = [c_int, i64, dbl, dp, dp]
    lib.o_scal.restype = None
    lib.o_asum.argtypes = [i64, dp, i64]
    lib.o_asum.restype = dbl
    _lib = lib
    return lib


def _arr(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


_PREC = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}


def prec_code(p) -> int:
    return _PREC[p]


def round_bf16(v: float) -> float:
    """Round an f32 value to bf16, nearest-even (NaN stays quiet NaN)."""
    return _load().o_round_bf16(float(v))


def scalar(prec, host: float, dev: float | None = None) -> float:
    """Effective scaling factor in the compute precision of ``prec``."""
    return _load().o_scalar(prec_code(prec), float(host), int(dev is not None),
                            0.0 if dev is None else float(dev))


def copy(y) -> np.ndarray:
    y = _arr(y)
    x = np.empty_like(y)
    _load().o_copy(y.size, _ptr(y), _ptr(x))
    return x


def axpby(prec, alpha: float, y, beta: float, z) -> np.ndarray:
    """x = RN(alpha*y + RN(beta*z)) elementwise; alpha, beta are effective factors."""
    y, z = _arr(y), _arr(z)
    assert y.size == z.size
    x = np.empty_like(y)
    _load().o_axpby(prec_code(prec), y.size, float(alpha), _ptr(y), float(beta), _ptr(z), _ptr(x))
    return x


def dot(x, y) -> float:
    x, y = _arr(x), _arr(y)
    assert x.size == y.size
    return _load().o_dot(x.size, _ptr(x), 1, _ptr(y), 1)


def nrm2(x) -> float:
    x = _arr(x)
    return _load().o_nrm2(x.size, _ptr(x))


def gemv(A, x, layout: int = ROW_MAJOR, trans: int = 0, m: int | None = None,
         n: int | None = None, lda: int | None = None) -> np.ndarray:
    """y = op(A) x.  ``A`` is either a 2-D array (m x n in its natural index
    order; its layout argument then says how it is laid out in memory) or a
    flat buffer with explicit m, n, lda."""
    A = np.asarray(A)
    if A.ndim == 2:
        m, n = A.shape
        flat = _arr(A.reshape(-1) if layout == ROW_MAJOR else A.T.reshape(-1))
        lda = n if layout == ROW_MAJOR else m
    else:
        flat = _arr(A)
        assert m is not None and n is not None and lda is not None
    x = _arr(x)
    out_len = n if trans else m
    assert x.size == (m if trans else n)
    y = np.empty(out_len, dtype=np.float64)
    if out_len:
        _load().o_gemv(layout, int(trans), m, n, _ptr(flat), lda, _ptr(x), _ptr(y))
    return y


def gemv_dot(prec, A, x, w, layout: int = ROW_MAJOR, trans: int = 0, m: int | None = None,
             n: int | None = None, lda: int | None = None):
    """(y, s): y = op(A) x as stored in ``prec`` ("f64" or "f32": the float64
    GEMV result, rounded to float32 for f32 storage), and s = <w, y> of that
    stored y.  Nothing but the two definitions in sequence."""
    if prec_code(prec) not in (F64, F32):
        raise ValueError("gemv_dot stores y in float64 or float32")
    y = gemv(A, x, layout, trans, m, n, lda)
    if prec_code(prec) == F32:
        y = y.astype(np.float32).astype(np.float64)  # round to nearest even
    return y, dot(w, y)


def _positions(n: int, inc: int) -> np.ndarray:
    """Buffer positions of the n logical elements of a strided vector, in the
    reference-BLAS convention: element i sits at i*inc for inc >= 0 and at
    (n-1-i)*|inc| for inc < 0 (a negative increment walks the buffer
    backwards from its end); inc == 0 repeats position 0."""
    i = np.arange(n, dtype=np.int64)
    return i * inc if inc >= 0 else (n - 1 - i) * (-inc)


def strided(buf, n: int, inc: int) -> np.ndarray:
    """The n logical elements of the strided vector (buf, inc)."""
    return np.asarray(buf, dtype=np.float64)[_positions(n, inc)]


def scatter(buf, vals, inc: int) -> np.ndarray:
    """A copy of ``buf`` with the logical elements of (buf, inc) replaced by
    ``vals``; every other entry is untouched."""
    out = np.array(buf, dtype=np.float64, copy=True)
    out[_positions(len(vals), inc)] = vals
    return out


def scal(prec, alpha: float, y) -> np.ndarray:
    """x = RN(alpha * y) elementwise; alpha is the effective factor."""
    y = _arr(y)
    x = np.empty_like(y)
    _load().o_scal(prec_code(prec), y.size, float(alpha), _ptr(y), _ptr(x))
    return x


def asum(x) -> float:
    x = _arr(x)
    return _load().o_asum(x.size, _ptr(x), 1)


def gemv_axpby(out_prec, alpha: float, A, x, beta: float, y, layout: int = ROW_MAJOR,
               trans: int = 0, m: int | None = None, n: int | None = None,
               lda: int | None = None) -> np.ndarray:
    """y <- alpha op(A) x + beta y with float64 or float32 output: the
    GEMV result rounded to ``out_prec`` (as stored), then
    RN(alpha s_i + RN(beta y_i)) in that precision -- or RN(alpha s_i) when
    beta == 0, where y is not read.  alpha and beta are rounded to the output
    precision first."""
    code = prec_code(out_prec)
    if code not in (F64, F32):
        raise ValueError("GEMV output is float64 or float32")
    s = gemv(A, x, layout, trans, m, n, lda)
    if code == F32:
        s = s.astype(np.float32).astype(np.float64)
    a = scalar(out_prec, alpha)
    if beta == 0.0:
        return scal(out_prec, a, s)
    return axpby(out_prec, a, s, scalar(out_prec, beta), _arr(y))


def ger(prec, u, v, layout: int = ROW_MAJOR, lda: int | None = None) -> np.ndarray:
    """A = u v^T with each entry rounded once to ``prec``.  Returns the flat
    buffer in ``layout`` order with leading dimension ``lda``."""
    u, v = _arr(u), _arr(v)
    m, n = u.size, v.size
    if lda is None:
        lda = n if layout == ROW_MAJOR else m
    lines = m if layout == ROW_MAJOR else n
    A = np.zeros(lines * lda, dtype=np.float64)
    _load().o_ger(prec_code(prec), layout, m, n, _ptr(u), _ptr(v), _ptr(A), lda)
    return A


def dot_backward(prec, zbar: float, x, y):
    """Gradient of z = <x, y> = sum_i x_i y_i: dz/dx_i = y_i and dz/dy_i = x_i,
    so with the upstream gradient zbar, dx_i = RN(zbar*y_i) and
    dy_i = RN(zbar*x_i): one IEEE product per element, rounded once to the
    storage precision (``scal``).  ``zbar`` is the effective factor in the
    compute precision.  Infinite, NaN and signed-zero entries scale as IEEE
    products do (zbar*inf = +-inf, -zbar * +0 = -0)."""
    return (scal(prec, zbar, y), scal(prec, zbar, x))


def gemv_backward(prec, A, x, ybar, layout: int = ROW_MAJOR):
    """Gradients of y = A x: dx = A^T ybar (reduction) and dA = ybar x^T."""
    dx = gemv(A, ybar, layout=layout, trans=1)
    dA = ger(prec, ybar, x, layout=layout)
    return dx, dA
