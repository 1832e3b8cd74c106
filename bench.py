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
events around each of its launches in the timed region, and the CPU oracle
timed on a bounded sample of the same workload.
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
DOMINANT_SOURCE = os.path.join(HERE, "paper_1409_0669_amd", "csrc", "gemv.hip")
TRAFFIC_FILE = os.path.join(HERE, "profiles", "gemv_rows_f64_16384_traffic.txt")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="time budget of the CPU oracle sample")
    ap.add_argument("--tuning", default=None, help="tuning table to load before timing")
    ap.add_argument("--settle", type=float, default=5.0,
                    help="seconds to wait before touching the GPU: for a few seconds after a process that "
                         "used tens of GB of device memory exits (the GPU test suite), HBM-bound kernels "
                         "run about 5 %% slower")
    ap.add_argument("--breakdown", action="store_true", help="print per-operation rates to stderr")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the adjoint, reduced-precision and composite rows")
    ap.add_argument("--kernel-profile", action="store_true",
                    help="run only the dominant kernel (GEMV 16384x16384 f64 row-major) and a calibration "
                         "copy of 2^26 f64 (512 MiB read, 512 MiB written), --steps times each, for "
                         "rocprofv3 kernel traces and counters")
    return ap.parse_args()


def kernel_profile(args, torch, W, ops):
    m = n = 16384
    A = W.device_draw(m * n, "f64", 0, 301).reshape(m, n)
    x = W.device_draw(n, "f64", 0, 401)
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    src = W.device_draw(1 << 26, "f64", 0, 501)
    dst = torch.empty_like(src)
    for name, fn in (("gemv_rows_f64_16384", lambda: ops.gemv(A, x, out=y)),
                     ("copy_f64_2^26", lambda: ops.copy(src, out=dst))):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        log("%-22s %d launches, %.1f us per launch (host clock)" % (name, args.steps,
                                                                   (time.perf_counter() - t0) * 1e6 / args.steps))


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
    """Device inputs of one step and the list of (name, bytes, callable)."""
    sizes = W.PAPER_SCALE["vector_sizes"]
    work = []
    keep = []
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
                         lambda y=y, z=z, x=x: ops.axpby(0.75, y, -1.25, z, out=x)))
            work.append((("dot", dt, n), 2 * n * s, lambda y=y, z=z, o=out_d: ops.dot(y, z, out=o)))
            work.append((("nrm2", dt, n), n * s, lambda y=y, o=out_n: ops.nrm2(y, out=o)))
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
    return work, keep


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
    outputs).  Returns (gemvs, dots, algorithmic bytes)."""
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
    return gemvs, dots, nbytes


def _replay_ms(torch, g, reps):
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def batched_rows(torch, W, ops, reps):
    """The uneven batch three ways: the batched plan (one launch, one
    work-group per work item) launched directly and replayed from its HIP
    graph, and -- as the baseline it replaces -- one library call per problem,
    all captured in one HIP graph."""
    from paper_1409_0669_amd.batch import BatchPlan
    out = {}
    for dt in ("bf16", "f32"):
        gemvs, dots, nbytes = uneven_batch(torch, W, ops, dt)
        plan = BatchPlan(gemvs, [(p, q, r) for p, q, r in dots], acc="compensated")
        ms = _median_ms(torch, plan.run, reps)
        info = plan.info()
        out["batched %s compensated, one launch (%d items)" % (dt, info["items"])] = {
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


def cpu_baseline(W, oracle, seconds):
    """The oracle (plain single-threaded C) on a bounded sample of the same
    workload: the vector operations at n = 1e5, 1e6, 1e7 and the 4096 x 4096
    matrix-vector products in both layouts, float32 and float64 values,
    repeated until the time budget is used."""
    import numpy as np
    items = []
    for dt in ("f32", "f64"):
        s = 4 if dt == "f32" else 8
        for i, n in enumerate((10 ** 5, 10 ** 6, 10 ** 7)):
            y = W.widen(W.quantize(W.uniform(n, 0, 100 + i), dt), dt)
            z = W.widen(W.quantize(W.uniform(n, 0, 200 + i), dt), dt)
            a, b = oracle.scalar(dt, 0.75), oracle.scalar(dt, -1.25)
            items.append((3 * n * s, lambda y=y, z=z, a=a, b=b, dt=dt: oracle.axpby(dt, a, y, b, z)))
            items.append((2 * n * s, lambda y=y, z=z: oracle.dot(y, z)))
            items.append((n * s, lambda y=y: oracle.nrm2(y)))
        m = n = 4096
        A = W.widen(W.quantize(W.uniform(m * n, 0, 300), dt), dt).reshape(m, n)
        xv = W.widen(W.quantize(W.uniform(n, 0, 400), dt), dt)
        At = np.ascontiguousarray(A.T).reshape(-1)
        nb = (m * n + m + n) * s
        items.append((nb, lambda A=A, x=xv: oracle.gemv(A, x)))
        items.append((nb, lambda F=At, x=xv: oracle.gemv(F, x, layout=oracle.COL_MAJOR, m=m, n=n, lda=m)))
    done_bytes, passes = 0, 0
    t0 = time.perf_counter()
    while True:
        for nb, fn in items:
            fn()
            done_bytes += nb
        passes += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt_s = time.perf_counter() - t0
    return {"value": round(done_bytes / dt_s / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "oracle (single-threaded C, fp64 Dot2 reductions) on axpby/dot/nrm2 at n=1e5,1e6,1e7 "
                      "and GEMV 4096x4096 row- and column-major, f32 and f64 values; %d passes in %.1f s"
                      % (passes, dt_s)}


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
    if args.settle > 0 and not args.kernel_profile:
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
    if args.kernel_profile:
        kernel_profile(args, torch, W, ops)
        return
    t0 = time.perf_counter()
    work, keep = build_workload(torch, W, ops)
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

    extra = None
    if not args.no_extra:
        log("timing the adjoint, reduced-precision and composite rows")
        extra = extra_rows(torch, W, ops, reps=max(5, args.steps))
        extra["step via HIP graph replay"] = graph_step(torch, work, max(5, args.steps))
        extra.update(batched_rows(torch, W, ops, max(5, args.steps // 2)))
        if args.breakdown:
            for k, v in extra.items():
                log("%-52s %s" % (k, v))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the CPU oracle sample (~%.0f s)" % args.cpu_seconds)
        cpu = cpu_baseline(W, oracle, args.cpu_seconds)

    line = {
        "metric": "achieved HBM GB/s (and % of peak) for axpy, dot, GEMV fwd/adjoint, plain vs batched/BF16",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "paper-scale plain kernels: axpby, dot, nrm2 at n=1e5,1e6,1e7,2^26 and GEMV "
                               "4096^2, 16384^2 row- and column-major; f32 and f64; uniform[-1,1) seed 0",
                   "bytes_per_step": step_bytes, "pct_of_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2)},
        "roofline": roofline, "cpu_baseline": cpu, "copy_ceiling": copy_ceiling, "breakdown_gbs": breakdown,
        "breakdown_gpu_gbs": breakdown_gpu,
        "cache_resident": cache_resident, "write_cached": write_cached, "other_rows": extra,
    }
    print(json.dumps(line), flush=True)
    del keep


if __name__ == "__main__":
    main()
