"""Benchmark of the bandwidth-limited BLAS-1/2 kernels on one MI355X.

One step is one pass over the paper-scale plain workload: for float32 and
float64 storage, the scaled vector addition x = a y + b z, the inner product and
the norm at n = 1e5, 1e6, 1e7 and 2^26, and the matrix-vector product y = A x
with A 4096 x 4096 and 16384 x 16384 in row- and column-major layout.  Inputs
are seeded synthetic data (uniform on [-1, 1)) resident in HBM before timing.

``value`` is the whole step's algorithmic bytes (minimal bytes: 3ns for the
addition, 2ns for the inner product, ns for the norm, (mn + m + n) elements for
the matrix-vector product) divided by the measured step time, in GB/s.
The JSON line also carries, for the dominant kernel (16384 x 16384 float64
row-major GEMV), its roofline against the 8 TB/s HBM peak measured with HIP
events around each of its launches in the timed region; the float64 part of
the step (and its HBM-resident part) as steps of their own; the small float64
set; the other rows of the hot path (adjoints, reduced precision, composites,
the uneven batch); and, after every GPU timing, the CPU leg: the oracle timed
on the whole step (with a naive multi-threaded float64 variant beside it, and
the host's core counts) and every result's error against the oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
MALL_BYTES = 256 * 1024 * 1024  # Infinity Cache of the MI355X
DOMINANT = ("gemv", "f64", "row", 16384)
AXPBY_ALPHA, AXPBY_BETA = 0.75, -1.25  # the step's scaled addition x = a y + b z
DOMINANT_SOURCE = os.path.join(HERE, "paper_1409_0669_amd", "csrc", "gemv.hip")
TRAFFIC_FILE = os.path.join(HERE, "profiles", "gemv_rows_f64_16384_traffic.txt")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU leg (the oracle and naive CPU timings and the accuracy report)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="least time of the oracle's passes over the step (the naive loops take half of it "
                         "per thread count)")
    ap.add_argument("--tuning", default=None, help="tuning table to load before timing")
    ap.add_argument("--accuracy-json", default=None,
                    help="also write the accuracy object (every row's error against the oracle) to this file")
    ap.add_argument("--settle", type=float, default=5.0,
                    help="seconds to wait before touching the GPU: for a few seconds after a process that "
                         "used tens of GB of device memory exits (the GPU test suite), HBM-bound kernels "
                         "run about 5 %% slower")
    ap.add_argument("--breakdown", action="store_true", help="print per-operation rates to stderr")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the adjoint, reduced-precision and composite rows")
    ap.add_argument("--kernel-profile", nargs="?", const="dominant", default=None,
                    choices=("dominant", "batch", "vectors", "adjoint"),
                    help="run only one group of kernels, --steps times each, for rocprofv3 kernel traces and "
                         "counters: 'dominant' = the GEMV 16384x16384 f64 row-major and a calibration copy of "
                         "2^26 f64 (512 MiB read, 512 MiB written); 'batch' = the uneven batch (bf16, f32, "
                         "compensated) and the standalone compensated GEMV 16384^2 of the same types; "
                         "'vectors' = axpby, copy, a write-only fill and dot at 2^26 f64; 'adjoint' = the "
                         "forward GEMV and dx = A^T ybar at the f32 differentiation shapes")
    return ap.parse_args()


def kernel_profile(args, torch, W, ops):
    """The kernels of one group launched back to back --steps times each
    (after --warmup calls), nothing else timed: input for rocprofv3."""
    def run(name, fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        log("%-40s %d launches, %.1f us per launch (host clock)" % (name, args.steps,
                                                                   (time.perf_counter() - t0) * 1e6 / args.steps))

    what = args.kernel_profile
    if what == "dominant":
        m = n = 16384
        A = W.device_draw(m * n, "f64", 0, 301).reshape(m, n)
        x = W.device_draw(n, "f64", 0, 401)
        y = torch.empty(m, dtype=torch.float64, device="cuda")
        src = W.device_draw(1 << 26, "f64", 0, 501)
        dst = torch.empty_like(src)
        run("gemv_rows_f64_16384", lambda: ops.gemv(A, x, out=y))
        run("copy_f64_2^26", lambda: ops.copy(src, out=dst))
    elif what == "batch":
        from paper_1409_0669_amd.batch import BatchPlan
        for dt in ("bf16", "f32"):
            gemvs, dots, nbytes, _ = uneven_batch(torch, W, ops, dt)
            plan = BatchPlan(gemvs, dots, acc="compensated")
            run("batch %s compensated (%.3f GB)" % (dt, nbytes / 1e9), plan.run)
            plan.close()
            del gemvs, dots
        for dt in ("bf16", "f32"):
            m = 16384
            A = W.device_draw(m * m, dt, 0, 912).view(m, m)
            x = W.device_draw(m, dt, 0, 913)
            y = torch.empty(m, dtype=torch.float32, device="cuda")
            run("gemv %s compensated 16384^2" % dt, lambda: ops.gemv(A, x, acc="compensated", out=y))
            del A
    elif what == "vectors":
        n = 1 << 26
        y = W.device_draw(n, "f64", 0, 1)
        z = W.device_draw(n, "f64", 0, 2)
        x = torch.empty_like(y)
        run("axpby f64 2^26", lambda: ops.axpby(0.75, y, -1.25, z, out=x))
        run("copy f64 2^26", lambda: ops.copy(y, out=x))
        run("fill f64 2^26 (torch, write only)", lambda: x.fill_(1.5))
        run("dot f64 2^26", lambda: ops.dot(y, z))
    else:
        for (m, n) in W.ADJOINT["gemv_shapes"]:
            A = W.device_draw(m * n, "f32", 0, 900).view(m, n)
            x = W.device_draw(n, "f32", 0, 901)
            yb = W.device_draw(m, "f32", 0, 902)
            y = torch.empty(m, dtype=torch.float32, device="cuda")
            dx = torch.empty(n, dtype=torch.float32, device="cuda")
            run("gemv fwd f32 %dx%d" % (m, n), lambda: ops.gemv(A, x, out=y))
            run("dx = A^T ybar f32 %dx%d" % (m, n), lambda: ops.gemv(A, yb, trans=True, out=dx))
            del A


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _write_cached(nbytes: int, written: int) -> bool:
    """True when a row's calls store a share of its bytes (at least 5 %) in an
    array that fits the Infinity Cache: timed back to back, those stores can
    stay in the cache instead of reaching HBM."""
    return 0 < written <= MALL_BYTES and written >= 0.05 * nbytes


def _step_written(name) -> int:
    """Bytes one step operation stores: the axpby's result vector (the
    reductions store one scalar, the GEMVs a vector below 0.1 % of their
    bytes)."""
    if name[0] != "axpby":
        return 0
    return name[2] * {"f32": 4, "f64": 8}[name[1]]


def build_workload(torch, W, ops):
    """Device inputs of one step, the list of (name, bytes, callable) and, per
    operation name, what the CPU leg needs to recompute it: its kind, storage
    type, input tensors and output tensor."""
    sizes = W.PAPER_SCALE["vector_sizes"]
    work = []
    keep = []
    specs = {}
    dev = "cuda"
    for dt in ("f32", "f64"):
        tdt = {"f32": torch.float32, "f64": torch.float64}[dt]
        s = 4 if dt == "f32" else 8
        for i, n in enumerate(sizes):
            y = W.device_draw(n, dt, 0, 100 + i)
            z = W.device_draw(n, dt, 0, 200 + i)
            x = torch.empty_like(y)
            out_d = torch.empty((), dtype=tdt, device=dev)
            out_n = torch.empty((), dtype=tdt, device=dev)
            keep += [y, z, x, out_d, out_n]
            work.append((("axpby", dt, n), 3 * n * s,
                         lambda y=y, z=z, x=x: ops.axpby(AXPBY_ALPHA, y, AXPBY_BETA, z, out=x)))
            work.append((("dot", dt, n), 2 * n * s, lambda y=y, z=z, o=out_d: ops.dot(y, z, out=o)))
            work.append((("nrm2", dt, n), n * s, lambda y=y, o=out_n: ops.nrm2(y, out=o)))
            specs[("axpby", dt, n)] = {"kind": "axpby", "dt": dt, "in": (y, z), "out": x}
            specs[("dot", dt, n)] = {"kind": "dot", "dt": dt, "in": (y, z), "out": out_d}
            specs[("nrm2", dt, n)] = {"kind": "nrm2", "dt": dt, "in": (y,), "out": out_n}
        for j, m in enumerate(W.PAPER_SCALE["gemv_shapes"]):
            m, n = m
            A_row = W.device_draw(m * n, dt, 0, 300 + j).reshape(m, n)
            A_col = A_row.t().contiguous().t()  # same matrix, column-major storage
            xv = W.device_draw(n, dt, 0, 400 + j)
            yv_r = torch.empty(m, dtype=tdt, device=dev)
            yv_c = torch.empty(m, dtype=tdt, device=dev)
            keep += [A_row, A_col, xv, yv_r, yv_c]
            nbytes = (m * n + m + n) * s
            work.append((("gemv", dt, "row", m), nbytes, lambda A=A_row, x=xv, y=yv_r: ops.gemv(A, x, out=y)))
            work.append((("gemv", dt, "col", m), nbytes, lambda A=A_col, x=xv, y=yv_c: ops.gemv(A, x, out=y)))
            # both layouts hold the same matrix: the CPU leg reads it row-major
            specs[("gemv", dt, "row", m)] = {"kind": "gemv", "dt": dt, "in": (A_row, xv), "out": yv_r}
            specs[("gemv", dt, "col", m)] = {"kind": "gemv", "dt": dt, "in": (A_row, xv), "out": yv_c}
    return work, keep, specs


def row_name(name) -> str:
    return "%s %s %s" % (name[0], name[1], "x".join(map(str, name[2:])))


class TimingEvent:
    """A HIP event for timing only, created with hipEventDisableSystemFence
    through the HIP runtime the process already uses.  Recording a default
    event ends with a system-scope fence (an L2 write-back and invalidate),
    which drains the queue and slows the kernel after it; an event without
    the fence timestamps the stream position and nothing else."""
    FLAGS = 0x20000000  # hipEventDefault | hipEventDisableSystemFence (timing enabled)
    _hip = None

    @classmethod
    def hip(cls):
        if cls._hip is None:
            import ctypes
            path = next(l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64.so" in l)
            h = ctypes.CDLL(path)
            h.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
            h.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            h.hipEventSynchronize.argtypes = [ctypes.c_void_p]
            h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
            h.hipEventDestroy.argtypes = [ctypes.c_void_p]
            cls._hip = h
        return cls._hip

    def __init__(self):
        import ctypes
        self.ev = ctypes.c_void_p()
        if self.hip().hipEventCreateWithFlags(ctypes.byref(self.ev), self.FLAGS) != 0:
            raise RuntimeError("hipEventCreateWithFlags failed")

    def record(self, stream):
        if self.hip().hipEventRecord(self.ev, stream) != 0:
            raise RuntimeError("hipEventRecord failed")

    def elapsed_ms(self, end):
        import ctypes
        t = ctypes.c_float()
        if self.hip().hipEventSynchronize(end.ev) != 0 or \
                self.hip().hipEventElapsedTime(ctypes.byref(t), self.ev, end.ev) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return t.value

    def __del__(self):
        if self._hip is not None and self.ev:
            self._hip.hipEventDestroy(self.ev)


def _median_ms(torch, fn, reps, batch=1, blocker=None):
    """Median over `reps` of the HIP-event interval around `batch` calls of
    fn launched back to back, divided by `batch`.  batch = 1 times a call
    alone: the GPU idles between calls, so the interval holds the dispatch
    latency of every launch.  A batch of calls overlaps each launch with the
    work before it, as in the timed step.  With a blocker (a long kernel of
    torch's own, enqueued before each interval) the calls are issued while
    the stream is still busy, so the interval holds the GPU's time for them
    rather than the host's time to issue them."""
    times = []
    fn()
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if blocker is not None:
            blocker()
        e0.record()
        for _ in range(batch):
            fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / batch)
    times.sort()
    return times[len(times) // 2]


PIPELINE = 8  # calls per timed interval for the per-operation rows


def extra_rows(torch, W, ops, reps):
    """The other rows of the hot path, each timed on its own (median of `reps`
    HIP-event intervals on the launch stream), outside the main metric:
    the copy, adjoint kernels at the differentiation shapes, reduced-precision
    storage with compensated accumulation, the composite operations and the
    BLAS-interface additions."""
    from paper_1409_0669_amd import composite
    out = {}

    def rate(name, nbytes, fn, written=0):
        # written: bytes each call stores.  When they fit the Infinity Cache,
        # back-to-back calls can keep the written array there, so the row is
        # flagged "write_cached" (its rate is not an HBM-roofline figure).
        ms = _median_ms(torch, fn, reps, batch=PIPELINE)
        alone = _median_ms(torch, fn, reps)
        out[name] = {"GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1), "us": round(ms * 1e3, 1),
                     "us_alone": round(alone * 1e3, 1)}
        if _write_cached(nbytes, written):
            out[name]["write_cached"] = True

    # adjoints (float32): y = A x, dx = A^T ybar, dA = ybar x^T; dot backward
    for (m, n) in W.ADJOINT["gemv_shapes"]:
        A = W.device_draw(m * n, "f32", 0, 900).view(m, n)
        x = W.device_draw(n, "f32", 0, 901)
        yb = W.device_draw(m, "f32", 0, 902)
        y = torch.empty(m, dtype=torch.float32, device="cuda")
        dx = torch.empty(n, dtype=torch.float32, device="cuda")
        dA = torch.empty_like(A)
        nb = (m * n + m + n) * 4
        rate("adjoint gemv fwd f32 %dx%d" % (m, n), nb, lambda: ops.gemv(A, x, out=y))
        rate("adjoint dx=A^T ybar f32 %dx%d" % (m, n), nb, lambda: ops.gemv(A, yb, trans=True, out=dx))
        rate("adjoint dA=ybar x^T f32 %dx%d" % (m, n), nb, lambda: ops.ger(yb, x, dA), written=m * n * 4)
        del A, dA
    nd = W.ADJOINT["dot_n"]
    xv = W.device_draw(nd, "f32", 0, 903)
    yv = W.device_draw(nd, "f32", 0, 904)
    zb = torch.tensor([0.37], dtype=torch.float32, device="cuda")
    gx, gy = torch.empty_like(xv), torch.empty_like(yv)
    rate("adjoint dot backward f32 n=2^24", 4 * nd * 4,
         lambda: (ops.scal_to(1.0, yv, out=gx, alpha_dev=zb), ops.scal_to(1.0, xv, out=gy, alpha_dev=zb)),
         written=2 * nd * 4)
    del xv, yv, gx, gy
    # the copy, the paper's calibration kernel and tuning proxy (x <- y, 2ns bytes)
    n = 1 << 26
    for dt in ("f64", "f32", "bf16"):
        s = {"f64": 8, "f32": 4, "bf16": 2}[dt]
        a = W.device_draw(n, dt, 0, 905)
        c = torch.empty_like(a)
        rate("copy %s n=2^26" % dt, 2 * n * s, lambda: ops.copy(a, out=c), written=n * s)
        del a, c
    # reduced precision: bf16 and f32 storage, float32 accumulation
    for dt in ("bf16", "f32"):
        s = 2 if dt == "bf16" else 4
        a = W.device_draw(n, dt, 0, 910)
        b = W.device_draw(n, dt, 0, 911)
        c = torch.empty_like(a)
        rate("precision axpby %s n=2^26" % dt, 3 * n * s, lambda: ops.axpby(0.75, a, -1.25, b, out=c), written=n * s)
        for acc in ("plain", "compensated"):
            rate("precision dot %s %s n=2^26" % (dt, acc), 2 * n * s, lambda acc=acc: ops.dot(a, b, acc=acc))
            rate("precision nrm2 %s %s n=2^26" % (dt, acc), n * s, lambda acc=acc: ops.nrm2(a, acc=acc))
        del a, b, c
        m = 16384
        A = W.device_draw(m * m, dt, 0, 912).view(m, m)
        x = W.device_draw(m, dt, 0, 913)
        y = torch.empty(m, dtype=torch.float32, device="cuda")
        for acc in ("plain", "compensated"):
            rate("precision gemv %s %s 16384^2" % (dt, acc), (m * m + 2 * m) * s,
                 lambda acc=acc: ops.gemv(A, x, acc=acc, out=y))
        del A
    # composite (float64, normal entries)
    n = W.COMPOSITE["n"]
    v = {k: W.device_draw(n, "f64", 0, 920 + i, dist="normal") for i, k in enumerate("xprq")}
    rate("composite cg step 3 calls n=2^24 (7n f64)", 7 * n * 8,
         lambda: composite.cg_step(1e-9, v["x"], v["p"], v["r"], v["q"]), written=2 * n * 8)
    rate("composite cg step fused n=2^24 (7n f64 of work)", 7 * n * 8,
         lambda: composite.cg_step_fused(1e-9, v["x"], v["p"], v["r"], v["q"]), written=2 * n * 8)
    del v
    m = W.COMPOSITE["gemv"][0]
    A = W.device_draw(m * m, "f64", 0, 930, dist="normal").view(m, m)
    pv = W.device_draw(m, "f64", 0, 931, dist="normal")
    q = torch.empty(m, dtype=torch.float64, device="cuda")
    rate("composite gemv 8192^2 + dot f64", (m * m + 3 * m) * 8, lambda: composite.gemv_dot(A, pv, q=q))
    rate("composite gemv 8192^2 + dot f64 fused epilogue (same work)", (m * m + 3 * m) * 8,
         lambda: composite.gemv_dot_fused(A, pv, q=q))
    del A
    # BLAS-interface additions (float64): scal and asum at unit increment;
    # strided vectors (bytes = the elements used, the lines in between are
    # fetched too); alpha/beta GEMV against the plain one
    n = 1 << 26
    a = W.device_draw(n, "f64", 0, 940)
    b = W.device_draw(n, "f64", 0, 941)
    rate("blas scal f64 n=2^26", 2 * n * 8, lambda: ops.scal(1.0000001, a), written=n * 8)
    for acc in ("plain", "compensated"):
        rate("blas asum f64 %s n=2^26" % acc, n * 8, lambda acc=acc: ops.asum(a, acc=acc))
    h = n // 2
    rate("blas dot f64 inc=2 n=2^25 (elements used)", 2 * h * 8, lambda: ops.dot(a[::2], b[::2]))
    rate("blas axpby f64 inc=2 n=2^25 (elements used)", 3 * h * 8,
         lambda: ops.axpby(0.5, a[::2], 0.25, b[::2], out=b[::2]))
    del a, b
    m = 16384
    A = W.device_draw(m * m, "f64", 0, 942).view(m, m)
    x = W.device_draw(m, "f64", 0, 943)
    y = W.device_draw(m, "f64", 0, 944)
    rate("blas gemv f64 16384^2 y = A x", (m * m + 2 * m) * 8, lambda: ops.gemv(A, x, out=y))
    rate("blas gemv f64 16384^2 y = 0.5 A x + 2 y", (m * m + 3 * m) * 8,
         lambda: ops.gemv(A, x, out=y, alpha=0.5, beta=2.0))
    del A
    return out


def uneven_batch(torch, W, ops, dtype):
    """The uneven batch: 512 row-major GEMVs with M, N log-uniform in
    [32, 4096] and 4096 dots with n log-uniform in [1e3, 1e6] (float32
    outputs).  Returns (gemvs, dots, algorithmic bytes, flat): flat holds the
    buffers the problems are views of, their offsets and sizes."""
    M, N, D = W.batched_sizes(0)
    s = 2 if dtype == "bf16" else 4
    align = 64

    def offsets(sizes):
        o, offs = 0, []
        for v in sizes:
            offs.append(o)
            o += (int(v) + align - 1) // align * align
        return offs, max(o, 1)
    a_off, a_tot = offsets(M * N)
    x_off, x_tot = offsets(N)
    d_off, d_tot = offsets(D)
    A = W.device_draw(a_tot, dtype, 0, 501)
    X = W.device_draw(x_tot, dtype, 0, 502)
    P = W.device_draw(d_tot, dtype, 0, 503)
    Q = W.device_draw(d_tot, dtype, 0, 504)
    Y = torch.empty(int(M.sum()), dtype=torch.float32, device="cuda")
    R = torch.empty(len(D), dtype=torch.float32, device="cuda")
    gemvs, dots, y0 = [], [], 0
    for i, (m, n) in enumerate(zip(M, N)):
        m, n = int(m), int(n)
        gemvs.append((A[a_off[i]:a_off[i] + m * n].view(m, n), X[x_off[i]:x_off[i] + n], Y[y0:y0 + m]))
        y0 += m
    for i, n in enumerate(D):
        n = int(n)
        dots.append((P[d_off[i]:d_off[i] + n], Q[d_off[i]:d_off[i] + n], R[i:i + 1]))
    nbytes = float(((M * N + M + N) * s).sum() + (2 * D * s).sum() + 4 * (M.sum() + len(D)))
    flat = {"A": A, "X": X, "P": P, "Q": Q, "Y": Y, "R": R, "a_off": a_off, "x_off": x_off, "d_off": d_off,
            "M": M, "N": N, "D": D}
    return gemvs, dots, nbytes, flat


def _replay_ms(torch, g, reps):
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def batched_rows(torch, W, ops, reps):
    """The uneven batch three ways: the batched plan (one launch per kind of
    work item, one work-group per item) launched directly and replayed from its HIP
    graph, and -- as the baseline it replaces -- one library call per problem,
    all captured in one HIP graph."""
    from paper_1409_0669_amd.batch import BatchPlan
    out = {}
    for dt in ("bf16", "f32"):
        gemvs, dots, nbytes, _ = uneven_batch(torch, W, ops, dt)
        plan = BatchPlan(gemvs, [(p, q, r) for p, q, r in dots], acc="compensated")
        ms = _median_ms(torch, plan.run, reps)
        info = plan.info()
        out["batched %s compensated, one plan run (%d items)" % (dt, info["items"])] = {
            "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 3), "bytes": int(nbytes)}
        cap = torch.cuda.Stream()
        plan.capture(cap)
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.replay()
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1))
        t.sort()
        out["batched %s compensated, plan graph replay" % dt] = {
            "GB/s": round(nbytes / (t[len(t) // 2] * 1e-3) / 1e9, 1), "ms": round(t[len(t) // 2], 3)}
        calls = [lambda A=A, x=x, y=y: ops.gemv(A, x, acc="compensated", out=y) for A, x, y in gemvs]
        calls += [lambda p=p, q=q, r=r: ops.dot(p, q, acc="compensated", out=r.view(())) for p, q, r in dots]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for c in calls:
                c()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for c in calls:
                c()
        ms = _replay_ms(torch, g, max(3, reps // 2))
        out["baseline %s: %d per-problem calls in one HIP graph" % (dt, len(calls))] = {
            "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 3)}
        plan.close()
        del gemvs, dots, g
    return out


def graph_step(torch, work, reps):
    """The same 32-operation step captured once in a HIP graph and replayed:
    the kernels are identical, launch overhead is removed."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            for _, _, fn in work:
                fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _, _, fn in work:
            fn()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    step_bytes = sum(b for _, b, _ in work)
    return {"GB/s": round(step_bytes / (ms * 1e-3) / 1e9, 1), "ms_per_step": round(ms, 4)}


# ---------------------------------------------------------------------------
# The CPU leg: the oracle on the step's own inputs (the CPU baseline), a naive
# multi-threaded float64 variant beside it, and every result's error against
# the oracle.  This leg is the only part of the benchmark that runs oracle/;
# it runs after every GPU timing and reads only the GPU outputs.
# ---------------------------------------------------------------------------
NAIVE_SRC = os.path.join(HERE, "bench_naive.c")
NAIVE_LIB = os.path.join(HERE, "bench_naive.so")
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5}  # the stated tolerances; 0 ULP for elementwise results


def build_naive(force: bool = False) -> str:
    """Compile bench_naive.c (plain loops, OpenMP) for any x86-64-v3 host."""
    if force or not os.path.exists(NAIVE_LIB) or os.path.getmtime(NAIVE_LIB) < os.path.getmtime(NAIVE_SRC):
        import subprocess
        tmp = NAIVE_LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, NAIVE_SRC,
                        "-lm"], check=True)
        os.replace(tmp, NAIVE_LIB)
    return NAIVE_LIB


def naive_lib():
    import ctypes
    lib = ctypes.CDLL(build_naive())
    dp, i64, dbl = ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_double
    lib.naive_axpby.argtypes = [i64, dbl, dp, dbl, dp, dp]
    lib.naive_axpby.restype = None
    lib.naive_dot.argtypes = [i64, dp, dp]
    lib.naive_dot.restype = dbl
    lib.naive_nrm2.argtypes = [i64, dp]
    lib.naive_nrm2.restype = dbl
    for f in (lib.naive_gemv_row, lib.naive_gemv_col):
        f.argtypes = [i64, i64, dp, i64, dp, dp]
        f.restype = None
    lib.naive_max_threads.restype = ctypes.c_int
    lib.naive_set_threads.argtypes = [ctypes.c_int]
    lib.naive_set_threads.restype = None
    return lib


def host_info() -> dict:
    """The host the CPU leg ran on: logical CPUs, the CPUs this process may
    use, and lscpu's model, sockets and physical cores."""
    import subprocess
    info = {"os_cpu_count": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        f = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f[k.strip()] = v.strip()
        info["model"] = f.get("Model name")
        sockets, per = int(f.get("Socket(s)", "0") or 0), int(f.get("Core(s) per socket", "0") or 0)
        info["sockets"], info["physical_cores"] = sockets, sockets * per
        info["threads_per_core"] = int(f.get("Thread(s) per core", "0") or 0)
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return info


# --- error measures ----------------------------------------------------------
def _ordered_bits(v, dt):
    """Integers in the order of the floating-point values of format dt, so
    that their difference counts units in the last place."""
    import numpy as np
    v = np.asarray(v, dtype=np.float64)
    if dt == "f64":
        b = v.view(np.int64)
        return np.where(b < 0, -(b & np.int64(0x7FFFFFFFFFFFFFFF)), b)
    b = v.astype(np.float32).view(np.int32).astype(np.int64)
    if dt == "bf16":
        b = b >> 16  # bf16 values are float32 values with 16 zero low bits
        return np.where(b < 0, -(b & 0x7FFF), b)
    return np.where(b < 0, -(b & 0x7FFFFFFF), b)


def err_elementwise(got, ref, dt) -> dict:
    import numpy as np
    d = np.abs(_ordered_bits(got, dt) - _ordered_bits(ref, dt))
    m = int(d.max()) if d.size else 0
    return {"max_ulp": m, "within_tol": m == 0}


def err_scalar(got, ref, dt, absum=None, cond=False) -> dict:
    """Relative error |got - ref| / |ref| and, for an inner product, the
    condition-scaled error |got - ref| / sum |x_i y_i|.  The bound is tol |ref|,
    or tol max(|ref|, sum |x_i y_i|) for plain float32 accumulation of f32 or
    bf16 data (cond)."""
    e = abs(float(got) - float(ref))
    r = {"rel": e / abs(ref) if ref else e}
    if absum is not None:
        r["cond"] = e / absum if absum else e
    scale = max(abs(ref), absum) if (cond and absum is not None) else abs(ref)
    r["within_tol"] = bool(e <= TOL[dt] * scale) if scale else e == 0.0
    return r


def err_gemv(got, ref, scale, dt) -> dict:
    """Componentwise max |y_i - y*_i| / (|A||x|)_i and normwise
    max |y - y*| / max |y*|; both within tol."""
    import numpy as np
    e = np.abs(np.asarray(got, dtype=np.float64) - ref)
    cw = float((e / np.maximum(scale, 1e-300)).max()) if e.size else 0.0
    rmax = float(np.abs(ref).max()) if e.size else 0.0
    nw = float(e.max()) / rmax if rmax else 0.0
    return {"componentwise": cw, "normwise": nw, "within_tol": bool(cw <= TOL[dt] and nw <= TOL[dt])}


def _max_err(rows) -> dict:
    """Largest value of each error measure over several problems."""
    out = {}
    for r in rows:
        for k, v in r.items():
            if k == "within_tol":
                out[k] = out.get(k, True) and v
            else:
                out[k] = max(out[k], v) if k in out else v
    return out


def cpu_leg(torch, W, ops, work, specs, seconds, extra=True):
    """(cpu_baseline, accuracy).  The oracle runs every operation of the step
    on the step's own inputs (float64 copies of the stored values), in step
    order, passes repeated until `seconds` have elapsed; the column-major
    products are evaluated on the row-major copy of the same matrix (the
    oracle's column-major walk would time the host's TLB, not its
    arithmetic).  The naive float64 loops then run the same passes on all the
    host's cores and on one.  The first oracle pass is also the reference
    for the accuracy of every step row."""
    import numpy as np

    import oracle
    cache = {}

    def host(t):
        if id(t) not in cache:
            cache[id(t)] = (t, W.from_torch(t, {torch.float64: "f64", torch.float32: "f32",
                                                  torch.bfloat16: "bf16"}[t.dtype]))
        return cache[id(t)][1]

    def oracle_op(sp):
        k, dt, xs = sp["kind"], sp["dt"], [host(t) for t in sp["in"]]
        if k == "axpby":
            return oracle.axpby(dt, oracle.scalar(dt, AXPBY_ALPHA), xs[0], oracle.scalar(dt, AXPBY_BETA), xs[1])
        if k == "dot":
            return oracle.dot(xs[0], xs[1])
        if k == "nrm2":
            return oracle.nrm2(xs[0])
        return oracle.gemv(xs[0], xs[1])

    t0 = time.perf_counter()
    for name, _, _ in work:  # download every input once, outside the timings
        for t in specs[name]["in"]:
            host(t)
    log("CPU leg: inputs on the host in %.1f s" % (time.perf_counter() - t0))
    step_bytes = sum(b for _, b, _ in work)
    refs, passes = {}, 0
    t0 = time.perf_counter()
    while True:
        for name, _, _ in work:
            r = oracle_op(specs[name])
            if passes == 0:
                refs[name] = r
        passes += 1
        if time.perf_counter() - t0 >= seconds:
            break
    t_or = time.perf_counter() - t0
    log("CPU leg: oracle, %d passes of the step in %.1f s" % (passes, t_or))

    lib = naive_lib()
    import ctypes
    dp = ctypes.POINTER(ctypes.c_double)
    ptr = lambda a: a.ctypes.data_as(dp)
    scratch = {}

    def naive_op(name):
        sp = specs[name]
        k, xs = sp["kind"], [host(t) for t in sp["in"]]
        if k == "axpby":
            o = scratch.setdefault(name, np.empty_like(xs[0]))
            lib.naive_axpby(xs[0].size, AXPBY_ALPHA, ptr(xs[0]), AXPBY_BETA, ptr(xs[1]), ptr(o))
        elif k == "dot":
            lib.naive_dot(xs[0].size, ptr(xs[0]), ptr(xs[1]))
        elif k == "nrm2":
            lib.naive_nrm2(xs[0].size, ptr(xs[0]))
        else:
            A, x = xs
            m, n = A.shape
            o = scratch.setdefault(name, np.empty(m))
            if name[2] == "row":
                lib.naive_gemv_row(m, n, ptr(A), n, ptr(x), ptr(o))
            else:  # the column-major product: the column sweep over A^T's storage
                At = scratch.get(("T", name[1], name[3]))
                if At is None:
                    At = scratch.setdefault(("T", name[1], name[3]), np.ascontiguousarray(A.T))
                lib.naive_gemv_col(m, n, ptr(At), m, ptr(x), ptr(o))

    for name, _, _ in work:  # column-major copies made outside the timing
        if name[0] == "gemv" and name[2] == "col":
            A = host(specs[name]["in"][0])
            scratch.setdefault(("T", name[1], name[3]), np.ascontiguousarray(A.T))
    naive = {}
    for threads in (max(1, int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))), 1):
        lib.naive_set_threads(threads)
        npass = 0
        t0 = time.perf_counter()
        while True:
            for name, _, _ in work:
                naive_op(name)
            npass += 1
            if time.perf_counter() - t0 >= seconds / 2:
                break
        dt_s = time.perf_counter() - t0
        naive[threads] = (round(step_bytes * npass / dt_s / 1e9, 3), npass, round(dt_s, 2))
        log("CPU leg: naive float64 loops, %d threads: %.2f GB/s" % (threads, naive[threads][0]))
    del scratch
    hi = host_info()
    many = max(naive)
    cpu = {"value": round(step_bytes * passes / t_or / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": "the whole step: every one of its %d operations (axpby, dot, nrm2 at n = 1e5, 1e6, 1e7, 2^26; "
                     "GEMV 4096^2 and 16384^2 in both layouts; f32 and f64 data held as float64) on the step's "
                     "own inputs, %d passes in %.1f s; single-threaded C, Dot2 reductions; the column-major "
                     "products on the row-major copy of the same matrix" % (len(work), passes, t_or),
           "host": hi,
           "naive_fp64": {"value": naive[many][0], "unit": "GB/s", "cores": many,
                          "passes": naive[many][1], "seconds": naive[many][2],
                          "kind": "plain float64 loops, OpenMP (bench_naive.c), the same passes"},
           "naive_fp64_1core": {"value": naive[1][0], "unit": "GB/s", "cores": 1, "passes": naive[1][1],
                                "seconds": naive[1][2]}}

    acc = {"tolerance": {"f64": TOL["f64"], "f32": TOL["f32"], "bf16": TOL["bf16"], "elementwise": "0 ULP"},
           "criteria": "elementwise: max ULP distance in the storage format; reductions: |got - ref| / |ref| "
                       "(rel), and / sum |x_i y_i| (cond) for inner products, bound tol |ref|, or tol "
                       "max(|ref|, sum |x_i y_i|) for plain float32 accumulation of f32/bf16 data; GEMV: "
                       "componentwise max |y_i - y*_i| / (|A||x|)_i and normwise max |y - y*| / max |y*|, both "
                       "within tol; ref = the oracle (Dot2, float64) on the stored inputs", "step": {}}
    for name, _, _ in work:
        sp = specs[name]
        got, ref, dt = W.from_torch(sp["out"], sp["dt"]), refs[name], sp["dt"]
        if sp["kind"] == "axpby":
            acc["step"][row_name(name)] = err_elementwise(got, ref, dt)
        elif sp["kind"] == "dot":
            y, z = (host(t) for t in sp["in"])
            acc["step"][row_name(name)] = err_scalar(float(got), ref, dt, float(np.abs(y * z).sum()),
                                                     cond=dt != "f64")
        elif sp["kind"] == "nrm2":
            acc["step"][row_name(name)] = err_scalar(float(got), ref, dt)
        else:
            A, x = (host(t) for t in sp["in"])
            acc["step"][row_name(name)] = err_gemv(got, ref, np.abs(A) @ np.abs(x), dt)
    cache.clear()
    refs.clear()
    if extra:
        t0 = time.perf_counter()
        acc.update(accuracy_extra(torch, W, ops, oracle))
        log("CPU leg: accuracy of the other rows in %.1f s" % (time.perf_counter() - t0))
    acc["all_within_tol"] = all(_all_within(v) for k, v in acc.items() if isinstance(v, dict) and k != "tolerance")
    return cpu, acc


def _all_within(d) -> bool:
    if "within_tol" in d:
        return bool(d["within_tol"])
    return all(_all_within(v) for v in d.values() if isinstance(v, dict))


def accuracy_extra(torch, W, ops, oracle) -> dict:
    """Each other row's error against the oracle: the small float64 set,
    adjoints, reduced precision (against the quantised inputs, and against
    the float64 draws before quantisation), composites, BLAS additions and
    every problem of the uneven batch.  Inputs are drawn as in the timed
    rows (same seeds); every operation runs once more here."""
    import numpy as np

    from paper_1409_0669_amd import autograd, composite
    h = lambda t, dt: W.from_torch(t, dt)
    out = {}
    # --- the small float64 set: axpby and dot at 2^20, GEMV 1024^2 row-major
    sm = W.SMALL_FP64
    n = sm["n"]
    y, z = W.device_draw(n, "f64", 0, 960), W.device_draw(n, "f64", 0, 961)
    y64, z64 = h(y, "f64"), h(z, "f64")
    row = {"axpby f64 n=2^20": err_elementwise(h(ops.axpby(AXPBY_ALPHA, y, AXPBY_BETA, z), "f64"),
                                               oracle.axpby("f64", AXPBY_ALPHA, y64, AXPBY_BETA, z64), "f64"),
           "dot f64 n=2^20": err_scalar(float(ops.dot(y, z).item()), oracle.dot(y64, z64), "f64",
                                        float(np.abs(y64 * z64).sum()))}
    m, k = sm["gemv"]
    A, x = W.device_draw(m * k, "f64", 0, 962).view(m, k), W.device_draw(k, "f64", 0, 963)
    A64, x64 = h(A, "f64"), h(x, "f64")
    row["gemv f64 1024^2 row-major"] = err_gemv(h(ops.gemv(A, x), "f64"), oracle.gemv(A64, x64),
                                                np.abs(A64) @ np.abs(x64), "f64")
    out["small_fp64_set"] = row
    # --- adjoints (float32): forward, dx = A^T ybar, dA = ybar x^T; dot backward
    adj = {}
    for (m, k) in W.ADJOINT["gemv_shapes"]:
        A = W.device_draw(m * k, "f32", 0, 900).view(m, k).requires_grad_(True)
        x = W.device_draw(k, "f32", 0, 901).requires_grad_(True)
        yb = W.device_draw(m, "f32", 0, 902)
        yv = autograd.gemv(A, x)
        yv.backward(yb)
        A64, x64, yb64 = h(A.detach(), "f32"), h(x.detach(), "f32"), h(yb, "f32")
        aA = np.abs(A64)
        adj["%dx%d" % (m, k)] = {
            "fwd": err_gemv(h(yv.detach(), "f32"), oracle.gemv(A64, x64), aA @ np.abs(x64), "f32"),
            "dx": err_gemv(h(x.grad, "f32"), oracle.gemv(A64, yb64, trans=1), aA.T @ np.abs(yb64), "f32"),
            "dA": err_elementwise(h(A.grad, "f32").reshape(-1), oracle.ger("f32", yb64, x64), "f32")}
        del A, x, yv, A64, aA
    nd = W.ADJOINT["dot_n"]
    xv = W.device_draw(nd, "f32", 0, 903).requires_grad_(True)
    yv = W.device_draw(nd, "f32", 0, 904).requires_grad_(True)
    zbar = torch.tensor(0.37, dtype=torch.float32, device="cuda")
    autograd.dot(xv, yv).backward(zbar)
    zb = oracle.scalar("f32", 1.0, float(zbar.item()))
    dxr, dyr = oracle.dot_backward("f32", zb, h(xv.detach(), "f32"), h(yv.detach(), "f32"))
    adj["dot backward n=2^24"] = _max_err([err_elementwise(h(xv.grad, "f32"), dxr, "f32"),
                                          err_elementwise(h(yv.grad, "f32"), dyr, "f32")])
    out["adjoint f32"] = adj
    del xv, yv
    # --- reduced precision: bf16 / f32 storage, float32 accumulation
    prec = {}
    n = 1 << 26
    for dt in ("bf16", "f32"):
        a, b = W.device_draw(n, dt, 0, 910), W.device_draw(n, dt, 0, 911)
        a64, b64 = h(a, dt), h(b, dt)
        af, bf = h(W.device_draw(n, "f64", 0, 910), "f64"), h(W.device_draw(n, "f64", 0, 911), "f64")
        ref, ref_full = oracle.dot(a64, b64), oracle.dot(af, bf)
        nref, nref_full = oracle.nrm2(a64), oracle.nrm2(af)
        absum = float(np.abs(a64 * b64).sum())
        for acc in ("plain", "compensated"):
            g = float(ops.dot(a, b, acc=acc).item())
            r = err_scalar(g, ref, dt, absum, cond=acc == "plain")
            r["rel_vs_fp64_draws"] = abs(g - ref_full) / abs(ref_full)
            prec["dot %s %s n=2^26" % (dt, acc)] = r
            g = float(ops.nrm2(a, acc=acc).item())
            r = err_scalar(g, nref, dt)
            r["rel_vs_fp64_draws"] = abs(g - nref_full) / abs(nref_full)
            prec["nrm2 %s %s n=2^26" % (dt, acc)] = r
        prec["axpby %s n=2^26" % dt] = err_elementwise(
            h(ops.axpby(AXPBY_ALPHA, a, AXPBY_BETA, b), dt),
            oracle.axpby(dt, oracle.scalar(dt, AXPBY_ALPHA), a64, oracle.scalar(dt, AXPBY_BETA), b64), dt)
        del a, b, a64, b64, af, bf
        m = 16384
        A, x = W.device_draw(m * m, dt, 0, 912).view(m, m), W.device_draw(m, dt, 0, 913)
        A64, x64 = h(A, dt), h(x, dt)
        ref, scale = oracle.gemv(A64, x64), np.abs(A64) @ np.abs(x64)
        del A64
        Af, xf = h(W.device_draw(m * m, "f64", 0, 912).view(m, m), "f64"), h(W.device_draw(m, "f64", 0, 913), "f64")
        ref_full = oracle.gemv(Af, xf)
        del Af
        for acc in ("plain", "compensated"):
            g = h(ops.gemv(A, x, acc=acc), "f32")
            r = err_gemv(g, ref, scale, dt)
            r["normwise_vs_fp64_draws"] = float(np.abs(g - ref_full).max() / np.abs(ref_full).max())
            prec["gemv %s %s 16384^2" % (dt, acc)] = r
        del A
    out["reduced_precision"] = prec
    # --- composites (float64, normal entries)
    comp = {}
    n = W.COMPOSITE["n"]
    v = {c: W.device_draw(n, "f64", 0, 920 + i, dist="normal") for i, c in enumerate("xprq")}
    hv = {c: h(t, "f64") for c, t in v.items()}
    a = 1e-9
    xr = oracle.axpby("f64", a, hv["p"], 1.0, hv["x"])
    rref = oracle.axpby("f64", -a, hv["q"], 1.0, hv["r"])
    rr = oracle.dot(rref, rref)
    for label, fn in (("3 calls", composite.cg_step), ("fused", composite.cg_step_fused)):
        x1, r1 = v["x"].clone(), v["r"].clone()
        g = float(fn(a, x1, v["p"], r1, v["q"]).item())
        comp["cg step n=2^24 %s" % label] = {"x": err_elementwise(h(x1, "f64"), xr, "f64"),
                                              "r": err_elementwise(h(r1, "f64"), rref, "f64"),
                                              "rr": err_scalar(g, rr, "f64")}
    del v, hv
    m = W.COMPOSITE["gemv"][0]
    A, p = W.device_draw(m * m, "f64", 0, 930, dist="normal").view(m, m), W.device_draw(m, "f64", 0, 931, dist="normal")
    A64, p64 = h(A, "f64"), h(p, "f64")
    qref, pqref = oracle.gemv_dot("f64", A64, p64, p64)
    scale = np.abs(A64) @ np.abs(p64)
    bound = 2.0 * float(np.abs(p64) @ scale)  # the GEMV bound carried through p, plus the inner product's
    for label, fn in (("two calls", composite.gemv_dot), ("fused epilogue", composite.gemv_dot_fused)):
        q, pq = fn(A, p)
        e = abs(float(pq.item()) - pqref)
        comp["gemv 8192^2 + dot %s" % label] = {
            "q": err_gemv(h(q, "f64"), qref, scale, "f64"),
            "pq": {"rel": e / abs(pqref), "vs_bound": e / bound, "within_tol": bool(e <= TOL["f64"] * bound)}}
    del A, A64
    out["composite f64"] = comp
    # --- BLAS additions (float64)
    blas = {}
    n = 1 << 26
    a, b = W.device_draw(n, "f64", 0, 940), W.device_draw(n, "f64", 0, 941)
    a64, b64 = h(a, "f64"), h(b, "f64")
    c = a.clone()
    ops.scal(1.0000001, c)
    blas["scal f64 n=2^26"] = err_elementwise(h(c, "f64"), oracle.scal("f64", 1.0000001, a64), "f64")
    del c
    for acc in ("plain", "compensated"):
        blas["asum f64 %s n=2^26" % acc] = err_scalar(float(ops.asum(a, acc=acc).item()), oracle.asum(a64), "f64")
    s2 = a64[::2] * b64[::2]
    blas["dot f64 inc=2 n=2^25"] = err_scalar(float(ops.dot(a[::2], b[::2]).item()), oracle.dot(a64[::2], b64[::2]),
                                              "f64", float(np.abs(s2).sum()))
    del a, b, a64, b64, s2
    m = 16384
    A, x, y = (W.device_draw(m * m, "f64", 0, 942).view(m, m), W.device_draw(m, "f64", 0, 943),
               W.device_draw(m, "f64", 0, 944))
    A64, x64, y64 = h(A, "f64"), h(x, "f64"), h(y, "f64")
    got = h(ops.gemv(A, x, out=y, alpha=0.5, beta=2.0), "f64")
    scale = 0.5 * (np.abs(A64) @ np.abs(x64)) + 2.0 * np.abs(y64)
    blas["gemv f64 16384^2 y = 0.5 A x + 2 y"] = err_gemv(got, oracle.gemv_axpby("f64", 0.5, A64, x64, 2.0, y64),
                                                          scale, "f64")
    del A, A64
    out["blas f64"] = blas
    # --- every problem of the uneven batch (compensated)
    from paper_1409_0669_amd.batch import BatchPlan
    for dt in ("bf16", "f32"):
        gemvs, dots, _, flat = uneven_batch(torch, W, ops, dt)
        plan = BatchPlan(gemvs, dots, acc="compensated")
        plan.run()
        torch.cuda.synchronize()
        Ah, Xh, Ph, Qh = (h(flat[k], dt) for k in ("A", "X", "P", "Q"))
        Yh, Rh = h(flat["Y"], "f32"), h(flat["R"], "f32")
        ge, de = [], []
        y0 = 0
        for i, (mm, nn) in enumerate(zip(flat["M"], flat["N"])):
            mm, nn = int(mm), int(nn)
            Ai = Ah[flat["a_off"][i]:flat["a_off"][i] + mm * nn].reshape(mm, nn)
            xi = Xh[flat["x_off"][i]:flat["x_off"][i] + nn]
            ge.append(err_gemv(Yh[y0:y0 + mm], oracle.gemv(Ai, xi), np.abs(Ai) @ np.abs(xi), dt))
            y0 += mm
        for i, nn in enumerate(flat["D"]):
            nn = int(nn)
            pi, qi = Ph[flat["d_off"][i]:flat["d_off"][i] + nn], Qh[flat["d_off"][i]:flat["d_off"][i] + nn]
            de.append(err_scalar(float(Rh[i]), oracle.dot(pi, qi), dt, float(np.abs(pi * qi).sum())))
        gm, dm = _max_err(ge), _max_err(de)
        out["batched %s compensated" % dt] = {
            "problems": len(ge) + len(de),
            "gemv_max": gm, "dot_max": dm,
            "within_tol": bool(gm.get("within_tol", True) and dm.get("within_tol", True))}
        plan.close()
        del gemvs, dots, flat, Ah, Xh, Ph, Qh
    return out


def subset_rate(torch, work, pick, steps) -> dict:
    """Several step operations (those `pick(name, bytes)` selects) launched
    back to back as their own step, `steps` times, timed as the main step."""
    sel = [(n, b, f) for n, b, f in work if pick(n, b)]
    for _, _, f in sel:
        f()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for _, _, f in sel:
            f()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nb = sum(b for _, b, _ in sel)
    gbs = nb * steps / el / 1e9
    return {"GB/s": round(gbs, 1), "pct_of_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
            "ms_per_step": round(el * 1e3 / steps, 4), "bytes_per_step": nb,
            "operations": [row_name(n) for n, _, _ in sel]}


def small_set_rows(torch, W, ops, reps) -> dict:
    """The small float64 set: axpby and dot at n = 2^20, GEMV 1024 x 1024
    row-major (uniform[-1, 1), seed 0).  Each row in GPU time (8 calls back to
    back behind a 2 GiB torch sum); every array fits the 256 MB Infinity
    Cache, so these are cache-resident rates, not HBM-roofline figures."""
    sm = W.SMALL_FP64
    n = sm["n"]
    y, z = W.device_draw(n, "f64", 0, 960), W.device_draw(n, "f64", 0, 961)
    x = torch.empty_like(y)
    o = torch.empty((), dtype=torch.float64, device="cuda")
    m, k = sm["gemv"]
    A, xv = W.device_draw(m * k, "f64", 0, 962).view(m, k), W.device_draw(k, "f64", 0, 963)
    yv = torch.empty(m, dtype=torch.float64, device="cuda")
    blk = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    out = {"cache_resident": True}
    for name, nb, fn in (("axpby f64 n=2^20", 3 * n * 8, lambda: ops.axpby(AXPBY_ALPHA, y, AXPBY_BETA, z, out=x)),
                         ("dot f64 n=2^20", 2 * n * 8, lambda: ops.dot(y, z, out=o)),
                         ("gemv f64 1024^2 row-major", (m * k + m + k) * 8, lambda: ops.gemv(A, xv, out=yv))):
        ms = _median_ms(torch, fn, reps, batch=PIPELINE, blocker=blk.sum)
        out[name] = {"GB/s": round(nb / (ms * 1e-3) / 1e9, 1), "us": round(ms * 1e3, 2), "bytes": nb}
    return out


def traffic_for_dominant():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if it was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    src_hash = hashlib.sha256(open(DOMINANT_SOURCE, "rb").read()).hexdigest()
    fields = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != src_hash:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    if args.settle > 0 and args.kernel_profile is None:
        time.sleep(args.settle)
    import torch
    import workloads as W
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(2)
    if args.tuning:
        ops.load_tuning(args.tuning)
    if args.kernel_profile is not None:
        kernel_profile(args, torch, W, ops)
        return
    t0 = time.perf_counter()
    work, keep, specs = build_workload(torch, W, ops)
    torch.cuda.synchronize()
    log("inputs ready in %.1f s (%d operations per step)" % (time.perf_counter() - t0, len(work)))

    step_bytes = sum(b for _, b, _ in work)
    for _ in range(args.warmup):
        for _, _, fn in work:
            fn()
    torch.cuda.synchronize()
    log("warmup done")

    # Timed region: K steps launched back to back; the only events in it
    # bracket each launch of the dominant kernel (created beforehand, timing
    # events without the system fence, recorded on the launch stream).
    dom_idx = next(i for i, (name, _, _) in enumerate(work) if name == DOMINANT)
    dom_ev = [(TimingEvent(), TimingEvent()) for _ in range(args.steps)]
    stream = torch.cuda.current_stream().cuda_stream
    fns = [fn for _, _, fn in work]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        for i, fn in enumerate(fns):
            if i == dom_idx:
                dom_ev[k][0].record(stream)
                fn()
                dom_ev[k][1].record(stream)
            else:
                fn()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = step_bytes * args.steps / elapsed / 1e9
    dom_each = [a.elapsed_ms(b) for a, b in dom_ev]
    dom_ms = sum(dom_each) / len(dom_each)
    log("dominant launch per step (us): " + " ".join("%.1f" % (t * 1e3) for t in dom_each))
    dom_bytes = work[dom_idx][1]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    cfg = ops.get_config(L.OP_GEMV_ROWS, torch.float64, DOMINANT[3], DOMINANT[3])
    kernel = "k_gemv_rows<double, %d, %d, %d, false>" % (cfg["vec"], cfg["rows"], cfg["unroll"])
    if cfg["split"] > 1:
        kernel += " + k_combine_lines (split %d)" % cfg["split"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for_dominant(),
                "kernel": kernel, "avg_launch_us": round(dom_ms * 1e3, 2), "algorithmic_bytes": dom_bytes}

    # Per-operation breakdown: a separate, untimed pass, each operation timed
    # on its own (median of HIP-event intervals around PIPELINE calls).
    breakdown = {}
    for name, nbytes, fn in work:
        ms = _median_ms(torch, fn, max(5, args.steps // 2), batch=PIPELINE)
        breakdown["%s %s %s" % (name[0], name[1], "x".join(map(str, name[2:])))] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    # The same rows in GPU time: each interval starts behind a 2 GiB torch
    # sum, so calls that the host issues more slowly than the GPU runs them
    # (the 1e5 and 1e6 rows) are timed by their kernels.
    blk = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    breakdown_gpu = {}
    for name, nbytes, fn in work:
        ms = _median_ms(torch, fn, max(5, args.steps // 2), batch=PIPELINE, blocker=blk.sum)
        breakdown_gpu["%s %s %s" % (name[0], name[1], "x".join(map(str, name[2:])))] = round(
            nbytes / (ms * 1e-3) / 1e9, 1)
    del blk
    if args.breakdown:
        for k, v in breakdown.items():
            log("%-28s %9.1f GB/s   GPU time %9.1f GB/s" % (k, v, breakdown_gpu[k]))
    # Rows whose working set fits the 256 MiB Infinity Cache: reported kernel
    # time only, no HBM-roofline claim.  Larger rows whose stored vector fits
    # it are listed apart: timed back to back, their stores can stay cached.
    cache_resident = ["%s %s %s" % (name[0], name[1], "x".join(map(str, name[2:])))
                      for name, nbytes, _ in work if nbytes < MALL_BYTES]
    write_cached = ["%s %s %s" % (name[0], name[1], "x".join(map(str, name[2:])))
                    for name, nbytes, _ in work
                    if nbytes >= MALL_BYTES and _write_cached(nbytes, _step_written(name))]
    # The measured copy ceiling (the paper's "achievable peak" next to the
    # specification): a 2^26-element f64 copy, timed as the breakdown.
    cy = W.device_draw(1 << 26, "f64", 0, 950)
    cx = torch.empty_like(cy)
    copy_gbs = 2 * (1 << 26) * 8 / (_median_ms(torch, lambda: ops.copy(cy, out=cx), max(5, args.steps),
                                                batch=PIPELINE) * 1e-3) / 1e9
    del cy, cx
    copy_ceiling = {"gbs": round(copy_gbs, 1), "value_frac": round(value / copy_gbs, 4),
                    "dominant_frac": round(achieved / copy_gbs, 4), "kernel": "k_copy f64 n=2^26"}
    # The paper's precision alone: the step's float64 operations as a step of
    # their own, and of those the ones whose arrays exceed the Infinity Cache
    # (2^26 vectors, 16384^2 matrices): the HBM-resident float64 part.
    f64_step = subset_rate(torch, work, lambda n, b: n[1] == "f64", args.steps)
    f64_hbm = subset_rate(torch, work, lambda n, b: n[1] == "f64" and b >= MALL_BYTES, args.steps)
    small = small_set_rows(torch, W, ops, max(5, args.steps))

    extra = None
    if not args.no_extra:
        log("timing the adjoint, reduced-precision and composite rows")
        extra = extra_rows(torch, W, ops, reps=max(5, args.steps))
        extra["step via HIP graph replay"] = graph_step(torch, work, max(5, args.steps))
        extra.update(batched_rows(torch, W, ops, max(5, args.steps // 2)))
        if args.breakdown:
            for k, v in extra.items():
                log("%-52s %s" % (k, v))

    cpu = accuracy = None
    if not args.no_cpu_baseline:
        log("CPU leg: the oracle and the naive loops on the step (~%.0f s each), then every row's error"
            % args.cpu_seconds)
        cpu, accuracy = cpu_leg(torch, W, ops, work, specs, args.cpu_seconds, extra=not args.no_extra)

    line = {
        "metric": "achieved HBM GB/s (and % of peak) for axpy, dot, GEMV fwd/adjoint, plain vs batched/BF16",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "paper-scale plain kernels: axpby, dot, nrm2 at n=1e5,1e6,1e7,2^26 and GEMV "
                               "4096^2, 16384^2 row- and column-major; f32 and f64; uniform[-1,1) seed 0",
                   "bytes_per_step": step_bytes, "pct_of_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2)},
        "roofline": roofline, "cpu_baseline": cpu, "copy_ceiling": copy_ceiling,
        "f64_step": f64_step, "f64_hbm_resident": f64_hbm, "small_fp64_set": small,
        "breakdown_gbs": breakdown, "breakdown_gpu_gbs": breakdown_gpu,
        "cache_resident": cache_resident, "write_cached": write_cached, "other_rows": extra,
        "accuracy": accuracy,
    }
    print(json.dumps(line), flush=True)
    if args.accuracy_json and accuracy is not None:
        with open(args.accuracy_json, "w") as f:
            json.dump({"device": torch.cuda.get_device_name(), "date": time.strftime("%Y-%m-%d"),
                       "command": "python bench.py --accuracy-json <file>", "accuracy": accuracy}, f, indent=1)
    del keep


if __name__ == "__main__":
    main()
