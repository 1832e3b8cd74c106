"""Host logic of the autotuner: the paper's configuration space and the
gfx950 candidate space (no GPU)."""
from __future__ import annotations

import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    d = {}
    for line in open(os.path.join(HERE, "golden", "paper_config_space.txt")):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        d[k.strip()] = v.split()
    return d


def test_paper_space_matches_the_paper():
    from paper_1409_0669_amd import tune
    g = _golden()
    sp = tune.paper_space()
    assert len(sp) == int(g["total"][0]) == 1900
    assert len(tune.PAPER_INCREMENTS) == int(g["increments"][0])
    assert len(tune.PAPER_VECTOR_TYPES) == int(g["vector_types"][0])
    assert len(tune.PAPER_LOCAL_SIZES) == int(g["local_sizes"][0])
    assert len(tune.PAPER_GROUPS) == int(g["work_group_counts"][0])
    assert tune.PAPER_LOCAL_SIZES[-1] == 512
    assert set(map(int, g["extra_work_group_counts"])) <= set(tune.PAPER_GROUPS)
    assert max(tune.PAPER_GROUPS) == 1024
    assert len({tuple(sorted(c.items())) for c in sp}) == 1900


def test_gfx950_space_is_valid_for_the_library():
    import ctypes
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import tune
    for cfg in tune.vector_space(256)[:200] + tune.rows_space()[:100] + tune.cols_space()[:100]:
        c = L.Config(**cfg)
        assert L.lib.bwla_set_config(L.OP_DOT, 0, -1, 3, ctypes.byref(c)) == L.OK, cfg
    L.lib.bwla_set_config(L.OP_DOT, 0, -1, -1, None)
    assert len(tune.vector_space(256)) == 5 * 5 * 3 * 2 * 7


def test_size_class_agrees_with_library():
    """The tuner's size classes are the library's: give every class its own
    block size and read back which one a call of a given size uses."""
    import ctypes
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import tune
    sizes = (0, (1 << 20) - 1, 1 << 20, (1 << 24) + 5, 1 << 28, (1 << 30) - 8, 1 << 30, 1 << 33)
    assert [tune.size_class(b) for b in sizes] == [0, 0, 1, 2, 3, 3, 4, 4]
    try:
        for k in range(5):
            assert L.lib.bwla_set_config(L.OP_COPY, L.F64, -1, k,
                                         ctypes.byref(L.Config(block=64 * (k + 1)))) == L.OK
        assert L.lib.bwla_set_config(L.OP_COPY, L.F64, -1, 5, ctypes.byref(L.Config(block=64))) == L.ERR_INVALID_ARG
        c = L.Config()
        for b in sizes:
            n = b // 16  # a copy streams 2 * 8 bytes per element
            assert L.lib.bwla_get_config(L.OP_COPY, L.F64, 0, 0, n, ctypes.byref(c)) == L.OK
            assert c.block == 64 * (tune.size_class(n * 16) + 1), b
    finally:
        L.lib.bwla_set_config(L.OP_COPY, L.F64, -1, -1, None)


def test_write_table_roundtrip(tmp_path):
    import ctypes
    import torch
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import tune
    p = str(tmp_path / "t.txt")
    tune.write_table([(L.OP_AXPBY, torch.float32, None, 3, dict(block=512, vec=8, unroll=2, grid=2048, increment=1)),
                      (L.OP_DOT, torch.float32, "plain", 3, dict(block=1024, vec=4, unroll=4, grid=256)),
                      (L.OP_DOT, torch.float32, "compensated", 3, dict(block=256, vec=4, unroll=2, grid=1024))], p)
    assert L.lib.bwla_load_tuning(p.encode()) == L.OK
    try:
        c = L.Config()
        for acc in (L.ACC_PLAIN, L.ACC_COMPENSATED):
            L.lib.bwla_get_config(L.OP_AXPBY, L.F32, acc, 0, 1 << 26, ctypes.byref(c))
            assert (c.block, c.vec, c.unroll, c.grid, c.increment) == (512, 8, 2, 2048, 1)
        L.lib.bwla_get_config(L.OP_DOT, L.F32, L.ACC_PLAIN, 0, 1 << 26, ctypes.byref(c))
        assert (c.block, c.unroll, c.grid) == (1024, 4, 256)
        L.lib.bwla_get_config(L.OP_DOT, L.F32, L.ACC_COMPENSATED, 0, 1 << 26, ctypes.byref(c))
        assert (c.block, c.unroll, c.grid) == (256, 2, 1024)
    finally:
        for op in (L.OP_AXPBY, L.OP_DOT):
            L.lib.bwla_set_config(op, L.F32, -1, -1, None)


def test_read_and_merge_tables(tmp_path):
    """A table read back equals what was written; merging replaces exactly
    the (op, dtype, acc, class) entries the new ones cover."""
    import torch
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import tune
    p = str(tmp_path / "t.txt")
    old = [(L.OP_AXPBY, torch.float32, None, 3, dict(block=512, vec=8, unroll=2, grid=2048, increment=1)),
           (L.OP_GEMV_COLS, torch.float32, "plain", 2, dict(block=512, vec=2, unroll=8, grid=256)),
           (L.OP_GEMV_COLS, torch.float32, "compensated", 2, dict(block=512, vec=2, unroll=8, grid=256)),
           (L.OP_GEMV_COLS, torch.float64, "plain", 2, dict(block=256, vec=2, unroll=4, grid=512))]
    tune.write_table(old, p)
    back = tune.read_table(p)
    assert [(o, d, a, c) for o, d, a, c, _ in back] == [(L.OP_AXPBY, L.F32, -1, 3), (L.OP_GEMV_COLS, L.F32, 0, 2),
                                                         (L.OP_GEMV_COLS, L.F32, 1, 2), (L.OP_GEMV_COLS, L.F64, 0, 2)]
    assert back[0][4] == dict(block=512, vec=8, unroll=2, grid=2048, increment=1, rows=0, split=0)
    new = [(L.OP_GEMV_COLS, torch.float32, "plain", 2, dict(block=1024, vec=1, unroll=8, grid=256))]
    merged = tune.merge_entries(back, new)
    tune.write_table(merged, p)
    rows = tune.read_table(p)
    keys = [(o, d, a, c) for o, d, a, c, _ in rows]
    assert keys == sorted(keys)                                     # written in key order
    got = {k: cfg for k, (_, _, _, _, cfg) in zip(keys, rows)}
    assert len(got) == 4
    assert got[(L.OP_GEMV_COLS, L.F32, 0, 2)]["block"] == 1024 and got[(L.OP_GEMV_COLS, L.F32, 0, 2)]["vec"] == 1
    assert got[(L.OP_GEMV_COLS, L.F32, 1, 2)]["block"] == 512       # the other mode is kept
    assert got[(L.OP_GEMV_COLS, L.F64, 0, 2)]["unroll"] == 4        # the other type is kept
    assert got[(L.OP_AXPBY, L.F32, -1, 3)]["increment"] == 1


def test_cols_candidates_include_one_element_per_lane():
    import torch
    from paper_1409_0669_amd import tune
    for dt, vecs in ((torch.float64, {1, 2}), (torch.float32, {1, 2, 4}), (torch.bfloat16, {1, 4, 8})):
        assert {c["vec"] for c in tune._cols_candidates(dt, False)} == vecs


def test_shipped_table_has_both_accumulation_modes():
    """The shipped table loads, and every reducing operation it tunes has an
    entry for each accumulation mode (elementwise operations: one shared)."""
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import tune
    rows = []
    for line in open(tune.DEFAULT_TABLE):
        line = line.split("#")[0].split()
        if line:
            assert len(line) == 11, line
            rows.append(tuple(int(v) for v in line))
    assert L.lib.bwla_load_tuning(tune.DEFAULT_TABLE.encode()) == L.OK
    reducing = {L.OP_DOT, L.OP_NRM2, L.OP_CG, L.OP_GEMV_ROWS, L.OP_GEMV_COLS, L.OP_BATCH}
    keys = {(op, t, a, k) for op, t, a, k, *_ in rows}
    for op, t, a, k, *_ in rows:
        if op in reducing:
            assert a in (0, 1) and (op, t, 1 - a, k) in keys, (op, t, a, k)
        else:
            assert a == -1, (op, t, a, k)


def test_study_analysis_on_synthetic_rates():
    """The configuration-study analysis: when every operation's rate is a fixed
    multiple of the copy's, the rank correlation is 1 and the copy's best
    configuration is every operation's best (no Table 2 penalty)."""
    import numpy as np
    from paper_1409_0669_amd import study, tune
    space = tune.vector_space(256)
    rng = np.random.default_rng(1)
    base = {study._key(c): float(rng.uniform(1000, 7000)) for c in space}
    rates = {op: {k: v * f for k, v in base.items()} for op, f in zip(study.OPS, (1.0, 0.9, 0.95, 0.8))}
    r = study.analyse(space, rates)
    assert r["n_configs"] == len(space)
    for op in study.OPS[1:]:
        assert abs(r["copy_vs_ops"][op]["spearman_rho"] - 1.0) < 1e-9
    for op in study.OPS:
        assert r["table2"][op]["with_copy_cfg"] == r["table2"][op]["own_best"]
    assert set(r["dot_distributions"]) == {"increment", "vec", "block", "grid"}
    md = study.markdown({"device": "synthetic", "cus": 256, "configs": len(space), "sizes": {"2000000": r}})
    assert "Table 2" in md and "Spearman" in md


def test_study_tie_band_penalty_range():
    """Two copy configurations tie (0.5 % apart): one is also the dot's best,
    the other costs the dot 40 %.  The argmax picks the first, the tie band
    shows the range 0 .. 40 % over both."""
    from paper_1409_0669_amd import study, tune
    space = tune.vector_space(256)[:50]
    keys = [study._key(c) for c in space]
    copy = {k: 1000.0 for k in keys}
    copy[keys[3]], copy[keys[7]] = 5000.0, 4975.0
    dot = {k: 900.0 for k in keys}
    dot[keys[3]], dot[keys[7]] = 3000.0, 5000.0
    rates = {"copy": copy, "axpby": dict(copy), "dot": dot, "nrm2": dict(copy)}
    r = study.analyse(space, rates)
    t2 = r["table2"]
    assert t2["config"] == dict(keys[3]) and t2["tie_configs"] == 2
    assert t2["dot"]["with_copy_cfg"] == round(3000 / 8000, 3)
    assert t2["dot"]["tie_penalty_pct"] == {"min": 0.0, "median": 20.0, "max": 40.0}
    assert t2["axpby"]["tie_penalty_pct"]["max"] == 0.5
    md = study.markdown({"device": "synthetic", "cus": 256, "configs": len(space), "sizes": {"67108864": r}})
    assert "0.0 / 20.0 / 40.0 %" in md and "within 2 % of the best copy" in md


def test_study_gemv_analysis_on_synthetic_rates():
    """GEMV part of the study: with the rate a known function of the
    configuration, the analysis finds the best configuration overall, the best
    with one row per work-group, and the paper's mapping at the copy's
    work-group size and vector width."""
    from paper_1409_0669_amd import study, tune
    space = tune.rows_space()
    rate = lambda c: 1000.0 + 100 * c["rows"] + 10 * c["vec"] + c["block"] / 1024 + (c["split"] == 1)
    rates = {study._key(c): rate(c) for c in space}
    g = study.analyse_gemv(space, rates, {"block": 256, "vec": 2, "unroll": 1, "grid": 0, "increment": 0})
    assert g["n_configs"] == len(space)
    assert g["own_best_config"]["rows"] == 8 and g["own_best_config"]["vec"] == 16
    assert g["one_row_per_group_best_config"]["rows"] == 1 and g["one_row_per_group_best_config"]["split"] == 1
    assert abs(g["copy_cfg_one_row_per_group"] - rate(dict(block=256, vec=2, rows=1, unroll=1, split=1)) / 8000) < 1e-3
    r = {"table2": {"config": {}, **{op: {"with_copy_cfg": 0.5, "own_best": 0.6} for op in study.OPS}},
         "copy_vs_ops": {}, "dot_distributions": {}, "gemv": dict(g, m=2048)}
    md = study.markdown({"device": "synthetic", "cus": 256, "configs": 1, "sizes": {"2000000": r}})
    assert "one row per work-group" in md and "2048 x 2048" in md


def test_multi_shape_pick_ranks_by_geometric_mean(monkeypatch):
    """A size class tuned on several shapes keeps the candidate whose
    geometric mean over the shapes is best, not the winner of one shape; the
    refinement re-times the leaders and can overturn the first ranking."""
    import torch
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import tune

    class FakeW:
        def __init__(self, name):
            self.name, self.table_op, self.dtype, self.cls, self.table_acc = name, L.OP_GEMV_ROWS, torch.float32, 2, "plain"
            self.bytes = 1e9

        def run(self):
            pass

    cands = [dict(block=256, grid=g) for g in (256, 512, 1024)]
    # first timing: the square shape loves grid 256, the tall one hates it
    first = {"square": {256: 7000.0, 512: 6000.0, 1024: 5000.0},
             "tall": {256: 1000.0, 512: 4000.0, 1024: 4500.0}}
    monkeypatch.setattr(tune, "sweep", lambda w, c, reps=6, log=None: sorted(
        ((cfg, 1.0, first[w.name][cfg["grid"]]) for cfg in c), key=lambda r: -r[2]))
    ws = [FakeW("square"), FakeW("tall")]
    cfg, score, rates = tune.multi_shape_pick(ws, cands, refine=0)
    # geometric means: 256 -> 2646, 512 -> 4899, 1024 -> 4743 (the square's winner comes last)
    assert cfg["grid"] == 512
    assert abs(score - (6000.0 * 4000.0) ** 0.5) < 1e-6 and rates == {0: 6000.0, 1: 4000.0}
    # with refinement the re-timed medians decide: make grid 1024 the clear winner
    current = {}
    monkeypatch.setattr(tune.ops, "set_config", lambda *a, **k: current.update(k))
    slow = {256: 2.0, 512: 0.5, 1024: 0.2}  # ms for 1 GB
    monkeypatch.setattr(tune, "time_ms", lambda fn, reps=10, warmup=2: slow[current["grid"]])
    cfg, score, rates = tune.multi_shape_pick(ws, cands, refine=3, refine_rounds=2)
    assert cfg["grid"] == 1024 and abs(score - 5000.0) < 1e-6 and len(rates) == 2


def test_workspace_size_cache_and_retry(monkeypatch):
    """ops caches workspace sizes, clears the cache when the configuration
    table changes through ops, and runs a call once more with a fresh size
    when the library reports the workspace too small (a table changed behind
    the cache)."""
    import torch
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops
    ops.reset_config()
    try:
        n = 1 << 22
        a = ops.workspace_size(L.OP_DOT, torch.float32, "plain", n=n)
        assert (L.OP_DOT, torch.float32, "plain", L.ROW_MAJOR, 0, 0, n, -1) in ops._ws_sizes
        ops.set_config(L.OP_DOT, torch.float32, -1, grid=65536)
        assert not ops._ws_sizes
        b = ops.workspace_size(L.OP_DOT, torch.float32, "plain", n=n)
        assert b >= 65536 * 16 > a
        # a size cached before a change made with the raw C call is stale: the
        # call is retried once with a fresh size
        ops.reset_config()
        ops.workspace_size(L.OP_DOT, torch.float32, "plain", n=n)
        L.lib.bwla_set_config(L.OP_DOT, L.F32, -1, -1, ctypes_config(L, grid=65536))
        sizes = []
        monkeypatch.setattr(ops, "workspace", lambda nbytes, device, stream=None: sizes.append(nbytes) or None)
        results = iter([L.ERR_WORKSPACE, L.OK])
        ops._with_workspace((L.OP_DOT, torch.float32, "plain", L.ROW_MAJOR, 0, 0, n), None, 0,
                            lambda ws, wsn: next(results))
        assert sizes[0] < sizes[1] and sizes[1] >= 65536 * 16
    finally:
        ops.reset_config()


def ctypes_config(L, **fields):
    import ctypes
    return ctypes.byref(L.Config(**fields))


def test_vector_sizes_cover_every_class_and_the_workload_lengths():
    """The tuned vector lengths include the paper-scale lengths and give every
    size class that a 2^16 .. 2^26 vector can fall in at least one length, for
    every operation and storage type."""
    import torch
    from paper_1409_0669_amd import tune
    for n in (10 ** 5, 10 ** 6, 10 ** 7, 1 << 26):
        assert n in tune.VEC_SIZES
    for es in (8, 4, 2):
        for per in (1, 2, 3, 6):
            tuned = {tune.size_class(per * es * n) for n in tune.VEC_SIZES}
            wanted = {tune.size_class(per * es * n) for n in range(1 << 16, (1 << 26) + 1, 1 << 14)}
            assert wanted <= tuned, (es, per, wanted - tuned)


def test_pick_from_sweeps_uses_every_length_of_a_class():
    """The entry of a class is the best geometric mean over its lengths, not
    the winner of the largest length."""
    import torch
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import tune

    class FakeW:
        table_op, dtype, cls, table_acc, bytes = L.OP_DOT, torch.float64, 1, "plain", 1e6

    a, b = dict(block=128, grid=1024), dict(block=512, grid=2048)
    small = [(a, 1.0, 900.0), (b, 1.0, 100.0)]
    large = [(b, 1.0, 5000.0), (a, 1.0, 4000.0)]
    cfg, score, rates = tune.pick_from_sweeps([FakeW(), FakeW()], [small, large], refine=0)
    assert cfg == a and rates == {0: 900.0, 1: 4000.0}


def test_time_ms_starts_each_interval_behind_the_blocker(monkeypatch):
    """While a blocker is set, every timed interval is opened after it, so
    the calls are issued while the stream is still busy; without one nothing
    runs before the interval."""
    from paper_1409_0669_amd import tune
    trace = []

    class FakeEvent:
        def __init__(self, enable_timing=False):
            self.t = None

        def record(self):
            trace.append("record")
            self.t = len(trace)

        def synchronize(self):
            pass

        def elapsed_time(self, other):
            return float(other.t - self.t)

    monkeypatch.setattr(tune.torch.cuda, "Event", FakeEvent)
    monkeypatch.setattr(tune, "_blocker", lambda: trace.append("block"))
    tune.time_ms(lambda: trace.append("call"), reps=2, warmup=1, batch=2)
    assert trace == ["call"] + ["block", "record", "call", "call", "record"] * 2
    trace.clear()
    monkeypatch.setattr(tune, "_blocker", None)
    tune.time_ms(lambda: trace.append("call"), reps=1, warmup=0, batch=1)
    assert trace == ["record", "call", "record"]


def test_batch_candidates_and_sizes():
    """The batch plans are tuned over work-group sizes up to 512 (the plans'
    limit) and packs per lane up to 32 (powers of two), on the uneven batch
    of 512 GEMVs and 4096 dots."""
    from paper_1409_0669_amd import tune
    for quick in (False, True):
        c = tune._batch_candidates(quick)
        assert c and all(d["block"] <= 512 and d["block"] % 64 == 0 for d in c)
        assert all(d["unroll"] in (1, 2, 4, 8, 16, 32) for d in c)
    M, N, D = tune._batch_sizes()
    assert len(M) == len(N) == 512 and len(D) == 4096
    assert "batch" in tune.ALL_OPS


def test_shipped_table_entries_come_from_the_committed_tuner_reports():
    """Every line of the shipped table is the class entry of a committed
    tuner run: the cols GEMV from its re-tune report, the batch plans from
    the batch report, every other operation from the full report."""
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    names = {0: "copy", 1: "axpby", 2: "dot", 3: "gemv_row", 4: "gemv_col", 5: "ger", 6: "nrm2", 7: "cg",
             8: "batch"}
    dts = {0: "f64", 1: "f32", 2: "bf16"}
    reports = {}
    for key, fname in (("full", "tuner_report_gfx950.json"), ("cols", "tuner_report_cols_gfx950.json"),
                       ("batch", "tuner_report_batch_gfx950.json")):
        with open(os.path.join(root, "results", fname)) as f:
            reports[key] = json.load(f)["results"]
    checked = 0
    with open(os.path.join(root, "paper_1409_0669_amd", "tuning", "gfx950.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            op, t, acc, cls, block, vec, unroll, grid, inc, rows, split = map(int, line.split())
            src = "cols" if op == 4 else "batch" if op == 8 else "full"
            acc_name = {-1: None, 0: "plain", 1: "compensated"}[acc]
            recs = [e for e in reports[src] if e["op"] == names[op] and e["dtype"] == dts[t] and e["class"] == cls
                    and (acc_name is None or e.get("acc") in (acc_name, None))]
            assert recs, line
            want = recs[0].get("class_entry") or recs[0]["best"]
            got = dict(block=block, vec=vec, unroll=unroll, grid=grid, increment=inc, rows=rows, split=split)
            assert all(got[k] == v for k, v in want.items() if k in got), (line, want)
            checked += 1
    assert checked >= 140
