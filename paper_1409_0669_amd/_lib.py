"""ctypes binding of ``libbwla.so`` (the C ABI in ``include/bwla.h``).

Argument marshalling only: every operation runs in the library's HIP kernels.
Importing this module fails loudly if the library has not been built; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# BWLA_LIBRARY may name another build of the same sources (the host-sanitizer
# build the CPU tests use); by default the in-tree library is loaded.
LIB_PATH = os.environ.get("BWLA_LIBRARY") or os.path.join(HERE, "libbwla.so")

# enums of bwla.h
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP, ERR_NOT_CAPTURABLE = range(6)
F64, F32, BF16 = 0, 1, 2
ROW_MAJOR, COL_MAJOR = 0, 1
ACC_PLAIN, ACC_COMPENSATED = 0, 1
INC_GLOBAL, INC_LOCAL = 0, 1
OP_COPY, OP_AXPBY, OP_DOT, OP_GEMV_ROWS, OP_GEMV_COLS, OP_GER, OP_NRM2, OP_CG, OP_BATCH = range(9)
OP_COUNT = 9
ABI_VERSION = 4  # BWLA_ABI_VERSION of include/bwla.h

STATUS_NAMES = {OK: "OK", ERR_INVALID_ARG: "INVALID_ARG", ERR_UNSUPPORTED: "UNSUPPORTED",
                ERR_WORKSPACE: "WORKSPACE", ERR_HIP: "HIP", ERR_NOT_CAPTURABLE: "NOT_CAPTURABLE"}

# Every function the header declares, with its ctypes signature.
vp, i64, i32, c_int, dbl, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                                ctypes.c_double, ctypes.c_size_t)


class Config(ctypes.Structure):
    _fields_ = [("block", i32), ("vec", i32), ("unroll", i32), ("grid", i32), ("increment", i32),
                ("rows", i32), ("split", i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GemvDesc(ctypes.Structure):
    _fields_ = [("A", vp), ("m", i64), ("n", i64), ("lda", i64), ("x", vp), ("y", vp)]


class DotDesc(ctypes.Structure):
    _fields_ = [("x", vp), ("y", vp), ("n", i64), ("out", vp)]


SIGNATURES = {
    "bwla_copy": (c_int, [c_int, i64, vp, vp, vp]),
    "bwla_axpby": (c_int, [c_int, i64, dbl, vp, vp, dbl, vp, vp, vp, vp]),
    "bwla_dot": (c_int, [c_int, c_int, i64, vp, vp, c_int, vp, vp, sz, vp]),
    "bwla_nrm2": (c_int, [c_int, c_int, i64, vp, c_int, vp, vp, sz, vp]),
    "bwla_dot_noalloc": (c_int, [c_int, c_int, i64, vp, vp, c_int, vp, vp]),
    "bwla_gemv": (c_int, [c_int, c_int, c_int, c_int, i64, i64, vp, i64, vp, c_int, vp, vp, sz, vp]),
    "bwla_gemv_dot": (c_int, [c_int, c_int, c_int, c_int, i64, i64, vp, i64, vp, vp, vp, c_int, vp, vp,
                              sz, vp]),
    "bwla_gemv_dot_workspace_size": (c_int, [c_int, c_int, c_int, i64, i64, ctypes.POINTER(sz)]),
    "bwla_copy_strided": (c_int, [c_int, i64, vp, i64, vp, i64, vp]),
    "bwla_axpby_strided": (c_int, [c_int, i64, dbl, vp, vp, i64, dbl, vp, vp, i64, vp, i64, vp]),
    "bwla_scal": (c_int, [c_int, i64, dbl, vp, vp, i64, vp]),
    "bwla_scal_to": (c_int, [c_int, i64, dbl, vp, vp, vp, vp]),
    "bwla_dot_strided": (c_int, [c_int, c_int, i64, vp, i64, vp, i64, c_int, vp, vp, sz, vp]),
    "bwla_nrm2_strided": (c_int, [c_int, c_int, i64, vp, i64, c_int, vp, vp, sz, vp]),
    "bwla_asum": (c_int, [c_int, c_int, i64, vp, i64, c_int, vp, vp, sz, vp]),
    "bwla_gemv_ex": (c_int, [c_int, c_int, c_int, c_int, i64, i64, dbl, vp, i64, vp, i64, dbl, c_int, vp, i64,
                             vp, sz, vp]),
    "bwla_gemv_ex_workspace_size": (c_int, [c_int, c_int, c_int, c_int, i64, i64, ctypes.POINTER(sz)]),
    "bwla_ger": (c_int, [c_int, c_int, i64, i64, vp, vp, vp, i64, vp]),
    "bwla_cg_update": (c_int, [c_int, c_int, i64, dbl, vp, vp, vp, vp, vp, c_int, vp, vp, sz, vp]),
    "bwla_workspace_size": (c_int, [c_int, c_int, c_int, c_int, c_int, i64, i64, ctypes.POINTER(sz)]),
    "bwla_batch_plan_create": (c_int, [c_int, c_int, c_int, ctypes.POINTER(GemvDesc), i32,
                                       ctypes.POINTER(DotDesc), i32, ctypes.POINTER(Config),
                                       ctypes.POINTER(vp)]),
    "bwla_batch_run": (c_int, [vp, vp]),
    "bwla_batch_capture": (c_int, [vp, vp]),
    "bwla_batch_replay": (c_int, [vp, vp]),
    "bwla_batch_info": (c_int, [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(dbl)]),
    "bwla_batch_plan_destroy": (None, [vp]),
    "bwla_set_config": (c_int, [c_int, c_int, c_int, c_int, ctypes.POINTER(Config)]),
    "bwla_get_config": (c_int, [c_int, c_int, c_int, i64, i64, ctypes.POINTER(Config)]),
    "bwla_load_tuning": (c_int, [ctypes.c_char_p]),
    "bwla_status_string": (ctypes.c_char_p, [c_int]),
    "bwla_last_error": (ctypes.c_char_p, []),
    "bwla_abi_version": (c_int, []),
    "bwla_device_cus": (c_int, []),
}


class BwlaError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))
        super().__init__("bwla %s: %s" % (self.status_name, message))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbwla.so is not built (expected at %s); build it with "
                          "`python -m paper_1409_0669_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.bwla_abi_version() != ABI_VERSION:
        raise ImportError("libbwla.so ABI version %d, expected %d" % (lib.bwla_abi_version(), ABI_VERSION))
    return lib


lib = _load()


def check(status: int) -> None:
    if status != OK:
        msg = lib.bwla_last_error()
        raise BwlaError(status, msg.decode() if msg else "")
