"""Bandwidth-limited linear algebra for AMD Instinct MI355X (gfx950).

The operations of Rupp et al., "Performance Portability Study of Linear Algebra
Kernels in OpenCL" (IWOCL 2014), Section 2 -- vector copy, scaled vector
addition, inner product and dense matrix-vector product -- plus the Euclidean
norm, gradients, batch plans for many uneven problems, fused composites
(a CG-style update, GEMV with an inner-product epilogue) and a BLAS-style
interface (increments, scal, asum, alpha/beta GEMV), as hand-written HIP
kernels behind the C ABI in ``include/bwla.h``.

Submodules (imported on first use; importing them fails loudly when
``libbwla.so`` has not been built):

* ``ops``       tensor-level calls (copy, axpby, scal, dot, nrm2, asum, gemv,
                gemv_dot, ger, cg_update)
* ``autograd``  ``GemvFn`` and ``DotFn`` with hand-written backward kernels
* ``batch``     ``BatchPlan``: many uneven GEMVs and dots, one launch per kind of
                work item, replayable from a HIP graph
* ``tune``      the autotuner and the configuration-space study
* ``build``     compiles the library with hipcc
"""
import importlib

_OPS = ("copy", "axpby", "scal", "dot", "nrm2", "asum", "gemv", "gemv_dot", "ger", "cg_update", "set_config",
        "get_config", "load_tuning", "reset_config", "BwlaError")


def __getattr__(name):
    if name in ("ops", "autograd", "batch", "composite", "tune", "study", "build", "_lib"):
        return importlib.import_module("." + name, __name__)
    if name in _OPS:
        return getattr(importlib.import_module(".ops", __name__), name)
    if name in ("GemvFn", "DotFn"):
        return getattr(importlib.import_module(".autograd", __name__), name)
    if name == "BatchPlan":
        return importlib.import_module(".batch", __name__).BatchPlan
    raise AttributeError(name)
