"""Autotuner and configuration-space study.

The paper (Section 2) defines a kernel configuration as the triple of
parameterised source, local work size and global work size, and sweeps four
axes: loop increment (global or local), vector type (double .. double16), local
work size (powers of two 1 .. 512) and number of work-groups (19 values) --
2 x 5 x 10 x 19 = 1900 configurations.  Its central claim (Section 3.2 and
Section 3.4, Table 2) is that configurations fast for the vector copy are fast
for the other bandwidth-bound operations, so one tuned configuration serves
them all.

This module re-derives that space for gfx950 (wave64, 256 CUs; work-group sizes
below 64 leave SIMD lanes idle, so local sizes run 64 .. 1024; the number of
work-groups is counted per CU; an "unroll" axis gives independent accesses in
flight), times every candidate with HIP events on the current stream, writes a
tuning table the C library loads (``bwla_load_tuning``), and reports the copy
proxy: each operation run with the copy's best configuration against its own
best (the Table 2 analogue).

The table has one entry per (operation, storage type, accumulation mode, size
class).  The reducing operations are tuned once per accumulation mode
(compensated arithmetic wants more waves in flight than plain).  Each size
class is tuned on every workload that falls in it -- vector lengths that are
powers of two and the paper-scale lengths 1e5, 1e6 and 1e7, GEMV shapes --
and keeps the candidate with the best geometric mean over them; a GEMV entry
is written as a work-group count, from which the library derives each shape's
split.
"""
from __future__ import annotations

import itertools
import json
import statistics
import time

import torch

from . import _lib as L
from . import ops

# ---- the paper's configuration space (Section 2) ---------------------------
PAPER_INCREMENTS = ("global", "local")
PAPER_VECTOR_TYPES = (1, 2, 4, 8, 16)
PAPER_LOCAL_SIZES = tuple(2 ** k for k in range(10))                     # 1 .. 512
PAPER_GROUPS = tuple(sorted(set(2 ** k for k in range(11)) | {48, 80, 96, 112, 160, 192, 224, 384}))


def paper_space():
    """All configurations of the paper's study, as dicts."""
    return [dict(increment=i, vector=v, local=l, groups=g)
            for i, v, l, g in itertools.product(PAPER_INCREMENTS, PAPER_VECTOR_TYPES,
                                                PAPER_LOCAL_SIZES, PAPER_GROUPS)]


# ---- the gfx950 space ------------------------------------------------------
BLOCKS = (64, 128, 256, 512, 1024)
VECS = (1, 2, 4, 8, 16)
UNROLLS = (1, 2, 4)
INCREMENTS = (L.INC_GLOBAL, L.INC_LOCAL)
GRID_PER_CU = (1, 2, 4, 8, 16, 32, 0)   # 0 = one pass: every thread does exactly `unroll` packs
ROWS = (1, 2, 4, 8)
SPLITS = (0, 1, 2, 4, 8, 16, 32)          # 0 = library heuristic


def vector_space(cus: int):
    """Candidate configurations of the streaming and reduction kernels."""
    out = []
    for b, v, u, inc, g in itertools.product(BLOCKS, VECS, UNROLLS, INCREMENTS, GRID_PER_CU):
        out.append(dict(block=b, vec=v, unroll=u, increment=inc, grid=g * cus))
    return out


def rows_space():
    return [dict(block=b, vec=v, rows=r, unroll=u, split=s)
            for b, v, r, u, s in itertools.product((64, 128, 256, 512, 1024), VECS, ROWS, (1, 2), SPLITS)]


def cols_space():
    return [dict(block=b, vec=v, unroll=u, split=s)
            for b, v, u, s in itertools.product((64, 128, 256, 512, 1024), VECS, UNROLLS, SPLITS)]


def size_class(nbytes: float) -> int:
    """Size class of the library's configuration table (bytes streamed)."""
    if nbytes < 1 << 20:
        return 0
    if nbytes < 1 << 24:
        return 1
    if nbytes < 1 << 28:
        return 2
    if nbytes < 1 << 30:
        return 3
    return 4


# ---- timing ----------------------------------------------------------------
PIPELINE = 4  # calls per timed interval


class _Blocker:
    """Keeps the stream busy while the calls under test are issued: a torch
    sum over a 2 GiB float64 buffer (a few hundred microseconds, reads only,
    and no kernel of this library, so no table entry changes its length).
    An interval that starts behind it holds the GPU's time for the calls
    alone.  Without it a small operation is timed at the host's rate of
    issuing calls (about 10 us each from Python), which hides every
    configuration whose kernels finish sooner."""

    def __init__(self, nbytes: int = 1 << 31):
        self.buf = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")

    def __call__(self):
        self.buf.sum()


_blocker = None  # a _Blocker while tune_all runs


def time_ms(fn, reps: int = 10, warmup: int = 2, batch: int = PIPELINE, blocked: bool = True) -> float:
    """Median duration of one fn() call: `reps` intervals, each bracketed by
    HIP events recorded on the current stream (the stream the library
    launches on) around `batch` calls launched back to back, divided by
    `batch`.  Back-to-back calls overlap each launch with the work before it,
    as a sequence of operations does; a call timed alone also holds the
    dispatch latency of an idle GPU (about 10 us), the same for every
    configuration.  While the tuner runs, each interval starts behind the
    blocker (see _Blocker), so it measures the GPU's time, not the host's."""
    for _ in range(warmup):
        fn()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if _blocker is not None and blocked:
            _blocker()
        e0.record()
        for _ in range(batch):
            fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / batch)
    return statistics.median(times)


# operations whose table entries are kept per accumulation mode
REDUCING = ("dot", "nrm2", "cg", "gemv", "batch")


class Workload:
    """Device operands of one tuned operation and its algorithmic bytes.  acc
    is the accumulation mode the reducing operations run with; the table
    entry they are tuned into is that mode's (elementwise operations have one
    entry for both modes)."""

    def __init__(self, op: str, dtype: torch.dtype, n: int = 0, m: int = 0, layout: str = "row",
                 acc: str = "plain"):
        import workloads as W
        self.op, self.dtype, self.n, self.m, self.layout = op, dtype, n, m, layout
        self.acc = acc
        self.table_acc = acc if op in REDUCING else None
        name = {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16"}[dtype]
        s = torch.tensor([], dtype=dtype).element_size()
        if op in ("copy", "axpby", "dot", "nrm2", "cg"):
            self.y = W.device_draw(n, name, 0, 1)
            self.z = W.device_draw(n, name, 0, 2)
            self.x = torch.empty_like(self.y)
            if op == "cg":
                self.r = W.device_draw(n, name, 0, 5)
                self.x.copy_(W.device_draw(n, name, 0, 6))
            self.bytes = {"copy": 2, "axpby": 3, "dot": 2, "nrm2": 1, "cg": 6}[op] * n * s
            self.table_op = {"copy": L.OP_COPY, "axpby": L.OP_AXPBY, "dot": L.OP_DOT, "nrm2": L.OP_NRM2,
                             "cg": L.OP_CG}[op]
        elif op == "ger":  # A <- u v^T, A m x n row-major
            self.A = torch.empty(m, n, dtype=dtype, device="cuda")
            self.u = W.device_draw(m, name, 0, 7)
            self.v = W.device_draw(n, name, 0, 8)
            self.bytes = (m * n + m + n) * s
            self.table_op = L.OP_GER
        elif op == "batch":  # the uneven batch: sizes (M[], N[], D[]) in `m`
            from .batch import BatchPlan
            Ms, Ns, Ds = m
            od = ops.default_out_dtype(dtype)
            # every problem starts 64 elements past the last (16-byte aligned
            # starts, as a caller's separate allocations would be)
            def offsets(sizes):
                o, offs = 0, []
                for v in sizes:
                    offs.append(o)
                    o += (int(v) + 63) // 64 * 64
                return offs, max(o, 1)
            a_off, a_tot = offsets([int(a) * int(b) for a, b in zip(Ms, Ns)])
            x_off, x_tot = offsets(Ns)
            d_off, d_tot = offsets(Ds)
            A = W.device_draw(a_tot, name, 0, 501)
            X = W.device_draw(x_tot, name, 0, 502)
            P = W.device_draw(d_tot, name, 0, 503)
            Q = W.device_draw(d_tot, name, 0, 504)
            self.gemvs = [(A[a_off[i]:a_off[i] + int(a) * int(b)].view(int(a), int(b)), X[x_off[i]:x_off[i] + int(b)],
                           torch.empty(int(a), dtype=od, device="cuda")) for i, (a, b) in enumerate(zip(Ms, Ns))]
            self.dots = [(P[d_off[i]:d_off[i] + int(d)], Q[d_off[i]:d_off[i] + int(d)],
                          torch.empty(1, dtype=od, device="cuda")) for i, d in enumerate(Ds)]
            self._plan_cls, self._plan, self._plan_cfg = BatchPlan, None, None
            self.bytes = int(BatchPlan(self.gemvs, self.dots, acc=acc).info()["bytes"])
            self.table_op = L.OP_BATCH
            self.table_acc = acc
        else:  # gemv_rows / gemv_cols: y = A x with A m x n in the layout that selects the kernel
            A = W.device_draw(m * n, name, 0, 3).view(m, n)
            self.A = A if layout == "row" else A.t().contiguous().t()
            self.x = W.device_draw(n, name, 0, 4)
            self.yv = torch.empty(m, dtype=ops.default_out_dtype(dtype), device="cuda")
            self.bytes = (m * n + m + n) * s
            self.table_op = L.OP_GEMV_ROWS if layout == "row" else L.OP_GEMV_COLS
        self.cls = size_class(self.bytes)

    def time(self, reps: int) -> float:
        """ms per call.  A batch plan (about a millisecond of GPU work in
        four launches) is timed as a single run on an idle stream, as the
        benchmark times it; behind the blocker, four runs back to back ranked
        its configurations differently from single runs."""
        if self.op == "batch":
            return time_ms(self.run, reps=reps, batch=1, blocked=False)
        return time_ms(self.run, reps=reps)

    def run(self):
        o = self.op
        if o == "copy":
            ops.copy(self.y, out=self.x)
        elif o == "axpby":
            ops.axpby(0.75, self.y, -1.25, self.z, out=self.x)
        elif o == "dot":
            ops.dot(self.y, self.z, acc=self.acc)
        elif o == "nrm2":
            ops.nrm2(self.y, acc=self.acc)
        elif o == "cg":
            # a tiny step keeps the iterates bounded over many repetitions
            ops.cg_update(1e-9, self.x, self.y, self.r, self.z, acc=self.acc)
        elif o == "ger":
            ops.ger(self.u, self.v, self.A)
        elif o == "batch":
            # a plan reads its configuration when it is built: rebuild it when
            # the table entry under test changes (in the untimed warm-up calls)
            cfg = ops.get_config(L.OP_BATCH, self.dtype, 0, self.bytes, acc=self.acc)
            if cfg != self._plan_cfg:
                self._plan = self._plan_cls(self.gemvs, self.dots, acc=self.acc)
                self._plan_cfg = cfg
            self._plan.run()
        else:
            ops.gemv(self.A, self.x, acc=self.acc, out=self.yv)


def _time_workload(w, reps: int) -> float:
    """ms per call of workload w: Workload.time for a batch plan, time_ms of
    its run otherwise."""
    if getattr(w, "op", None) == "batch":
        return w.time(reps)
    return time_ms(w.run, reps=reps)


def sweep(w: Workload, candidates, reps: int = 8, log=None, refine: int = 0, refine_rounds: int = 5):
    """Time every candidate configuration on workload w.  Returns a list of
    (config, ms, GB/s) sorted by speed.

    With refine = k > 0 the k fastest are timed again, round-robin over
    `refine_rounds` rounds of `reps` runs each, and ranked by the median of all
    their runs: the fastest of hundreds of short measurements is partly
    noise, and interleaving spreads any drift of the device over all k."""
    res = []
    for cfg in candidates:
        ops.set_config(w.table_op, w.dtype, w.cls, acc=w.table_acc, **cfg)
        try:
            ms = _time_workload(w, reps)
        except L.BwlaError as e:  # e.g. a configuration the shape cannot use
            if log:
                log("skip %s: %s" % (cfg, e))
            continue
        res.append((cfg, ms, w.bytes / (ms * 1e-3) / 1e9))
    res.sort(key=lambda r: r[1])
    if refine > 1 and len(res) > 1:
        top = [r[0] for r in res[:refine]]
        runs = {i: [] for i in range(len(top))}
        for _ in range(refine_rounds):
            for i, cfg in enumerate(top):
                ops.set_config(w.table_op, w.dtype, w.cls, acc=w.table_acc, **cfg)
                runs[i].append(_time_workload(w, reps))
        again = sorted(((top[i], statistics.median(t), w.bytes / (statistics.median(t) * 1e-3) / 1e9)
                        for i, t in runs.items()), key=lambda r: r[1])
        res = again + res[refine:]
    ops.set_config(w.table_op, w.dtype, w.cls, acc=w.table_acc)
    return res


ACC_CODE = {None: -1, "plain": L.ACC_PLAIN, "compensated": L.ACC_COMPENSATED}


def write_table(entries, path: str) -> None:
    """entries: list of (op code, dtype, acc, size class, config dict); acc is
    "plain", "compensated" or None (both modes share the entry)."""
    code = {torch.float64: L.F64, torch.float32: L.F32, torch.bfloat16: L.BF16}
    with open(path, "w") as f:
        f.write("# bwla tuning table: op dtype acc size_class block vec unroll grid increment rows split\n")
        f.write("# written %s on %s\n" % (time.strftime("%Y-%m-%d %H:%M:%S"),
                                          torch.cuda.get_device_name() if torch.cuda.is_available() else "?"))
        for op, dt, acc, cls, c in entries:
            f.write("%d %d %d %d %d %d %d %d %d %d %d\n" % (
                op, code[dt], ACC_CODE[acc], cls, c.get("block", 0), c.get("vec", 0), c.get("unroll", 0),
                c.get("grid", 0), c.get("increment", 0), c.get("rows", 0), c.get("split", 0)))


def copy_proxy(results: dict) -> dict:
    """results: {op: [(cfg, ms, GB/s), ...]} over the same vector candidate
    list.  For each op, the rate of the copy's best configuration and of the
    op's own best (the paper's Table 2 comparison)."""
    best_copy = results["copy"][0][0]
    key = json.dumps(best_copy, sort_keys=True)
    rep = {"copy_best": best_copy}
    for op, res in results.items():
        own = res[0]
        with_copy = next((r for r in res if json.dumps(r[0], sort_keys=True) == key), None)
        rep[op] = {"own_best": own[0], "own_best_gbs": round(own[2], 1),
                   "with_copy_cfg_gbs": round(with_copy[2], 1) if with_copy else None,
                   "penalty_pct": round(100 * (1 - with_copy[2] / own[2]), 2) if with_copy else None}
    return rep


# ---- the tuning run -------------------------------------------------------
# Vector lengths tuned: powers of two spanning the size classes and the
# lengths of the paper-scale workload (1e5, 1e6, 1e7); each class entry is
# picked over every length that falls in the class.
VEC_SIZES = (1 << 16, 10 ** 5, 10 ** 6, 1 << 20, 10 ** 7, 1 << 23, 1 << 25, 1 << 26)

import os as _os

DEFAULT_TABLE = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "tuning", "gfx950.txt")
_DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def _vector_candidates(dtype, cus, quick, reduction=False):
    """Streaming candidates; reductions also try eight packs in flight and
    eight work-groups per CU (more bytes in flight for a single stream)."""
    native = 16 // torch.tensor([], dtype=dtype).element_size()
    vecs = (native,) if quick else (max(1, native // 2), native, min(16, 2 * native))
    blocks = (256, 1024) if quick else (128, 256, 512, 1024)
    unrolls = (1, 2, 4, 8) if reduction else (1, 2, 4)
    grids = (1, 2, 4, 8, 0) if reduction else (1, 2, 4, 0)
    return [dict(block=b, vec=v, unroll=u, increment=i, grid=g * cus)
            for b in blocks for v in vecs for u in unrolls for i in (0, 1) for g in grids]


# GEMV candidates name a work-group count (per CU; 0 = the library's
# heuristic) rather than a split: the library turns it into the split of each
# shape, so one candidate means the same on a square, a tall and a wide matrix
GEMV_GROUPS_PER_CU = (0, 1, 2, 4, 8, 16, 32, 64)


def _rows_candidates(dtype, quick, cus=256):
    native = 16 // torch.tensor([], dtype=dtype).element_size()
    vecs = (native,) if quick else (max(1, native // 2), native)
    return [dict(block=b, vec=v, rows=r, unroll=u, split=0, grid=g * cus) for b in (256, 512, 1024) for v in vecs
            for r in (1, 2, 4, 8) for u in (1, 2) for g in GEMV_GROUPS_PER_CU]


def _cols_candidates(dtype, quick, cus=256):
    # one element per lane included: with few outputs the cols kernel's
    # split (and its second kernel) grows with the pack width
    # 16 and 32 lines in flight only where the library takes them (at most 128
    # bytes of A per lane in flight)
    es = torch.tensor([], dtype=dtype).element_size()
    native = 16 // es
    vecs = (native,) if quick else tuple(sorted({1, max(1, native // 2), native}))
    return [dict(block=b, vec=v, unroll=u, split=0, grid=g * cus) for b in (256, 512, 1024) for v in vecs
            for u in (2, 4, 8, 16, 32) if u <= 8 or u * v * es <= 128 for g in GEMV_GROUPS_PER_CU]


# GEMV shapes tuned; each size class is tuned on every shape that falls in it
# (the square matrices of the paper-scale workload and the tall and wide
# shards of the differentiation workload)
GEMV_SHAPES = ((1024, 1024), (4096, 4096), (16384, 2048), (2048, 16384), (8192, 8192), (16384, 16384))


def multi_shape_pick(workloads, candidates, reps=6, refine=6, refine_rounds=5, log=None):
    """The candidate with the best geometric mean of GB/s over several
    workloads (shapes of one size class, all with the same table entry).
    Every candidate is timed once per workload, then ranked as in
    :func:`pick_from_sweeps`.  Returns (best config, score in GB/s,
    {workload index: GB/s of the best})."""
    sweeps = [sweep(w, candidates, reps=reps, log=log) for w in workloads]
    return pick_from_sweeps(workloads, sweeps, reps=reps, refine=refine, refine_rounds=refine_rounds)


def pick_from_sweeps(workloads, sweeps, reps=6, refine=6, refine_rounds=5):
    """Rank the candidates that every sweep timed (sweeps[i] is a list of
    (config, ms, GB/s) for workloads[i]) by the geometric mean of their GB/s
    over the workloads; the `refine` best are timed again round-robin over
    `refine_rounds` rounds and ranked by the geometric mean of their medians.
    Returns (best config, score in GB/s, {workload index: GB/s of the best})."""
    keyf = lambda c: json.dumps(c, sort_keys=True)
    per = [{keyf(c): (c, g) for c, _, g in res} for res in sweeps]
    common = [k for k in per[0] if all(k in p for p in per[1:])]

    def gmean(vals):
        return float(statistics.geometric_mean(vals))

    ranked = sorted(common, key=lambda k: -gmean([p[k][1] for p in per]))
    top = ranked[:max(1, refine)]
    if refine > 1 and len(top) > 1:
        runs = {k: [[] for _ in workloads] for k in top}
        for _ in range(refine_rounds):
            for k in top:
                for i, w in enumerate(workloads):
                    ops.set_config(w.table_op, w.dtype, w.cls, acc=w.table_acc, **per[0][k][0])
                    runs[k][i].append(_time_workload(w, reps))
        w0 = workloads[0]
        ops.set_config(w0.table_op, w0.dtype, w0.cls, acc=w0.table_acc)
        rate = {k: [w.bytes / (statistics.median(runs[k][i]) * 1e-3) / 1e9 for i, w in enumerate(workloads)]
                for k in top}
        best = max(top, key=lambda k: gmean(rate[k]))
        return per[0][best][0], gmean(rate[best]), dict(enumerate(rate[best]))
    best = ranked[0]
    return per[0][best][0], gmean([p[best][1] for p in per]), {i: p[best][1] for i, p in enumerate(per)}


def _ger_candidates(dtype, quick):
    native = 16 // torch.tensor([], dtype=dtype).element_size()
    return [dict(block=b, vec=v, rows=r) for b in (128, 256, 512, 1024)
            for v in (max(1, native // 2), native, min(16, 2 * native)) for r in (1, 2, 4, 8)]


def _batch_candidates(quick):
    # the work-group size and the packs of a GEMV row each lane of a staged
    # tile owns (fewer packs: more lanes share a row)
    return [dict(block=b, unroll=u) for b in ((256, 512) if quick else (128, 256, 512))
            for u in ((8, 16) if quick else (4, 8, 16, 32))]


# the uneven batch tuned on: 512 GEMVs with M, N log-uniform in [32, 4096] and
# 4096 dots with n log-uniform in [1e3, 1e6], seed 0
def _batch_sizes():
    import workloads as W
    return W.batched_sizes(0)


# what tune_all can tune; "gemv_row" / "gemv_col" are the rows and cols GEMV
# kernels, "batch" the batch plans
ALL_OPS = ("copy", "axpby", "dot", "nrm2", "cg", "gemv_row", "gemv_col", "ger", "batch")


def tune_all(dtypes=("f64", "f32", "bf16"), quick=False, log=print, ops_=ALL_OPS, vec_sizes=None,
             gemv_shapes=None, ger_shapes=None, max_candidates=None, accs=("plain", "compensated"),
             batch_sizes=None):
    """Sweep every operation of `ops_`, storage type, accumulation mode (for
    the reducing operations, of `accs`) and size class; return the table
    entries and a report (best and default rates, copy proxy).  vec_sizes,
    gemv_shapes and ger_shapes replace the workloads tuned on;
    max_candidates keeps only the first candidates of each list (both for a
    quick check of the tuner itself, not for a table); batch_sizes (M[], N[],
    D[]) replaces the uneven batch."""
    global _blocker
    _blocker = _Blocker()
    try:
        return _tune_all(dtypes, quick, log, ops_, vec_sizes or VEC_SIZES, gemv_shapes or GEMV_SHAPES,
                         ger_shapes or ((4096, 4096), (16384, 16384)), max_candidates, accs,
                         batch_sizes or _batch_sizes())
    finally:
        _blocker = None


def _tune_all(dtypes, quick, log, ops_, vec_sizes, gemv_shapes, ger_shapes, max_candidates, accs, batch_sizes):
    cut = (lambda c: c[:max_candidates]) if max_candidates else (lambda c: c)
    cus = L.lib.bwla_device_cus()
    ops.reset_config()
    entries, report = [], {"device": torch.cuda.get_device_name(), "cus": cus, "results": [], "copy_proxy": {},
                           "timing": "GPU time: each interval starts behind a 2 GiB torch sum"}
    refine = 0 if quick else 6

    def record(w, res, default_ms, **where):
        rec = {"op": w.op if w.op != "gemv" else "gemv_" + w.layout, "dtype": where.pop("dn"),
               "acc": w.table_acc, "class": w.cls, "bytes": w.bytes, "best": res[0][0],
               "best_gbs": round(res[0][2], 1), "default_gbs": round(w.bytes / (default_ms * 1e-3) / 1e9, 1)}
        rec.update(where)
        report["results"].append(rec)
        log("%-9s %-4s %-11s %-13s class %d best %7.1f GB/s default %7.1f GB/s %s" % (
            rec["op"], rec["dtype"], w.table_acc or "", "x".join(str(v) for v in where.values()), w.cls,
            res[0][2], rec["default_gbs"], res[0][0]))

    for dn in dtypes:
        dt = _DT[dn]
        cands = cut(_vector_candidates(dt, cus, quick))
        cands_red = cut(_vector_candidates(dt, cus, quick, reduction=True))
        proxy_in = {}
        es = torch.tensor([], dtype=dt).element_size()
        for op in ("copy", "axpby", "dot", "nrm2", "cg"):
            if op not in ops_:
                continue
            per_elem = {"copy": 2, "axpby": 3, "dot": 2, "nrm2": 1, "cg": 6}[op] * es
            by_class = {}
            for n in vec_sizes:
                by_class.setdefault(size_class(per_elem * n), []).append(n)
            for acc in (accs if op in REDUCING else ("plain",)):
                for cls, sizes in sorted(by_class.items()):
                    # the workloads of one class live together: the pick re-times the leaders on each
                    ws, sweeps, recs = [], [], []
                    for n in sizes:
                        w = Workload(op, dt, n=n, acc=acc)
                        default_ms = time_ms(w.run, reps=10)
                        res = sweep(w, cands_red if op in ("dot", "nrm2") else cands, reps=6, refine=refine)
                        record(w, res, default_ms, dn=dn, n=n)
                        recs.append(report["results"][-1])
                        if n == vec_sizes[-1] and op != "cg" and acc == "plain":
                            proxy_in[op] = res
                        ws.append(w)
                        sweeps.append(res)
                    cfg, score, rates = pick_from_sweeps(ws, sweeps, refine=refine)
                    for i, rec in enumerate(recs):
                        rec["class_entry"], rec["class_entry_gbs"] = cfg, round(rates[i], 1)
                    log("%-9s %-4s %-11s class %d entry over n=%s: %s, %s GB/s" % (
                        op, dn, acc if op in REDUCING else "", cls, ",".join(str(n) for n in sizes), cfg,
                        [round(rates[i], 1) for i in range(len(ws))]))
                    entries.append((Workload_table_op(op), dt, acc if op in REDUCING else None, cls, cfg))
                    del ws, sweeps
        if "copy" in proxy_in:
            report["copy_proxy"][dn] = copy_proxy(proxy_in)
        by_class = {}
        for (m, n) in gemv_shapes:
            by_class.setdefault(size_class((m * n + m + n) * es), []).append((m, n))
        for layout, cands_g in (("row", cut(_rows_candidates(dt, quick, cus))),
                                ("col", cut(_cols_candidates(dt, quick, cus)))):
            if "gemv_" + layout not in ops_:
                continue
            for acc in accs:
                for cls, shapes in sorted(by_class.items()):
                    ws = [Workload("gemv", dt, n=n, m=m, layout=layout, acc=acc) for (m, n) in shapes]
                    default = [w.bytes / (time_ms(w.run, reps=10) * 1e-3) / 1e9 for w in ws]
                    cfg, score, rates = multi_shape_pick(ws, cands_g, refine=refine)
                    entries.append((ws[0].table_op, dt, acc, cls, cfg))
                    rec = {"op": "gemv_" + layout, "dtype": dn, "acc": acc, "class": cls, "shapes": shapes,
                           "best": cfg, "best_gbs_per_shape": [round(rates[i], 1) for i in range(len(ws))],
                           "best_gbs_geomean": round(score, 1), "default_gbs_per_shape": [round(d, 1) for d in default]}
                    report["results"].append(rec)
                    log("gemv_%-4s %-4s %-11s class %d %-40s best %s GB/s default %s GB/s %s" % (
                        layout, dn, acc, cls, " ".join("%dx%d" % sh for sh in shapes), rec["best_gbs_per_shape"],
                        rec["default_gbs_per_shape"], cfg))
                    del ws
        for (m, n) in (ger_shapes if "ger" in ops_ else ()):
            w = Workload("ger", dt, n=n, m=m)
            default_ms = time_ms(w.run, reps=10)
            res = sweep(w, cut(_ger_candidates(dt, quick)), reps=6, refine=refine)
            entries.append((L.OP_GER, dt, None, w.cls, res[0][0]))
            record(w, res, default_ms, dn=dn, m=m, n=n)
            del w
        if "batch" in ops_:
            for acc in accs:
                w = Workload("batch", dt, m=batch_sizes, acc=acc)
                default_ms = w.time(10)
                res = sweep(w, cut(_batch_candidates(quick)), reps=6, refine=refine)
                entries.append((L.OP_BATCH, dt, acc, w.cls, res[0][0]))
                record(w, res, default_ms, dn=dn, gemvs=len(batch_sizes[0]), dots=len(batch_sizes[2]))
                del w
    return entries, report


def Workload_table_op(op: str) -> int:
    return {"copy": L.OP_COPY, "axpby": L.OP_AXPBY, "dot": L.OP_DOT, "nrm2": L.OP_NRM2, "cg": L.OP_CG}[op]


def read_table(path: str):
    """The entries of a tuning table as (op, dtype code, acc code, class,
    config dict) tuples (the format write_table writes)."""
    out = []
    for line in open(path):
        line = line.split("#", 1)[0].split()
        if len(line) != 11:
            continue
        v = [int(t) for t in line]
        out.append((v[0], v[1], v[2], v[3], dict(zip(("block", "vec", "unroll", "grid", "increment", "rows",
                                                      "split"), v[4:]))))
    return out


def merge_entries(old, new_entries):
    """old: read_table() rows; new_entries: tune_all() entries.  Returns
    write_table() entries: the old ones, with every (op, dtype, acc, class)
    that the new ones cover replaced, ordered by that key."""
    code = {torch.float64: L.F64, torch.float32: L.F32, torch.bfloat16: L.BF16}
    dt_of = {v: k for k, v in code.items()}
    acc_of = {v: k for k, v in ACC_CODE.items()}
    key = lambda op, dtc, accc, cls: (op, dtc, accc, cls)
    covered = {key(op, code[dt], ACC_CODE[acc], cls) for op, dt, acc, cls, _ in new_entries}
    kept = [(op, dt_of[dtc], acc_of[accc], cls, cfg) for op, dtc, accc, cls, cfg in old
            if key(op, dtc, accc, cls) not in covered]
    merged = kept + list(new_entries)
    order = lambda e: (e[0], code[e[1]], ACC_CODE[e[2]], e[3])
    return sorted(merged, key=order)


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="tune the bwla kernels on this GPU")
    ap.add_argument("--out", default=DEFAULT_TABLE, help="tuning table to write")
    ap.add_argument("--report", default=None, help="JSON report to write")
    ap.add_argument("--dtypes", default="f64,f32,bf16")
    ap.add_argument("--ops", default=",".join(ALL_OPS), help="operations to tune: " + ",".join(ALL_OPS))
    ap.add_argument("--merge", default=None,
                    help="a table whose other entries are kept (the tuned ones are replaced)")
    ap.add_argument("--quick", action="store_true", help="smaller candidate lists")
    args = ap.parse_args(argv)
    sel = tuple(args.ops.split(","))
    bad = [o for o in sel if o not in ALL_OPS]
    if bad:
        ap.error("unknown operations %s" % bad)
    t0 = time.time()
    old = read_table(args.merge) if args.merge else None  # before --out may overwrite it
    entries, report = tune_all(tuple(args.dtypes.split(",")), quick=args.quick,
                               log=lambda *a: print(*a, flush=True), ops_=sel)
    if old is not None:
        entries = merge_entries(old, entries)
    _os.makedirs(_os.path.dirname(_os.path.abspath(args.out)), exist_ok=True)
    write_table(entries, args.out)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    print("wrote %s (%d entries) in %.0f s" % (args.out, len(entries), time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
