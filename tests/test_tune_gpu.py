"""The autotuner itself on the GPU: a short run (two candidates per
operation, small sizes) must time its candidates, write a table the library
loads, and the operations must stay within the oracle's criteria when run
with that table."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.criteria import TOL, check_scalar, check_vector, cond_scale
from tests.gpu_util import host, mat, need_gpu, vec

pytestmark = pytest.mark.gpu


def test_tuner_smoke_writes_a_table_the_library_uses(tmp_path):
    need_gpu()
    import torch
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd import ops, tune
    ops.reset_config()
    try:
        bsizes = (np.array([37, 300, 5]), np.array([1000, 64, 3000]), np.array([5000, 70000, 1]))
        entries, report = tune.tune_all(("f32",), quick=True, log=lambda *a: None,
                                        ops_=("dot", "gemv_row", "gemv_col", "batch"), vec_sizes=(1 << 16, 1 << 18),
                                        gemv_shapes=((512, 384),), max_candidates=2, accs=("plain",),
                                        batch_sizes=bsizes)
        kinds = {(op, cls) for op, _, _, cls, _ in entries}
        assert (L.OP_DOT, 0) in kinds and (L.OP_DOT, 1) in kinds
        assert {op for op, _, _, _, _ in entries} == {L.OP_DOT, L.OP_GEMV_ROWS, L.OP_GEMV_COLS, L.OP_BATCH}
        assert all(r.get("best_gbs", r.get("best_gbs_geomean", 0)) > 0 for r in report["results"])
        path = str(tmp_path / "table.txt")
        tune.write_table(entries, path)
        ops.load_tuning(path)
        for op, _, acc, cls, cfg in entries:  # the library now resolves the tuned entries
            if op == L.OP_DOT and cls == 1:  # 2^18 f32 elements of two vectors: 2 MiB
                got = ops.get_config(L.OP_DOT, torch.float32, 0, 1 << 18)
                assert (got["block"], got["unroll"]) == (cfg["block"], cfg["unroll"])
        for n in (1 << 16, 100_003, 1 << 18):
            x, x64 = vec(n, "f32", 1700)
            y, y64 = vec(n, "f32", 1701)
            check_scalar(float(ops.dot(x, y).item()), oracle.dot(x64, y64),
                         cond_scale("f32", "plain", np.abs(x64 * y64).sum()), TOL["f32"], "dot %d" % n)
        for layout in ("row", "col"):
            A, A64 = mat(512, 384, "f32", 1702, layout=layout)
            xv, xv64 = vec(384, "f32", 1703)
            check_vector(host(ops.gemv(A, xv)), oracle.gemv(A64, xv64), np.abs(A64) @ np.abs(xv64), TOL["f32"],
                         "gemv " + layout)
        # a batch plan built under the tuned batch entry
        from paper_1409_0669_amd.batch import BatchPlan
        from tests.batch_util import check, from_sizes
        (bcfg,) = [cfg for op, _, _, _, cfg in entries if op == L.OP_BATCH]
        gemvs, dots = from_sizes("f32", *bsizes, seed=4)
        nbytes = BatchPlan(gemvs, dots).info()["bytes"]
        got = ops.get_config(L.OP_BATCH, torch.float32, 0, int(nbytes))
        assert (got["block"], got["unroll"]) == (bcfg["block"], bcfg["unroll"])
        BatchPlan(gemvs, dots).run()
        torch.cuda.synchronize()
        check("f32", "plain", gemvs, dots)
    finally:
        ops.reset_config()
        ops.load_default_tuning()


def test_configuration_study_on_a_small_space(monkeypatch):
    """The configuration study end to end on the GPU, over a few
    configurations of each space and small sizes: it times every operation
    in every configuration, analyses the rates into the report (distributions,
    copy against the other operations, the single-configuration comparison,
    the GEMV part) and renders it; the shipped table is restored after."""
    need_gpu()
    from paper_1409_0669_amd import ops, study, tune
    vfull, rfull = tune.vector_space, tune.rows_space
    vsub = lambda cus: vfull(cus)[::150]
    rsub = lambda: [c for c in rfull() if c["block"] == 256 and c["unroll"] == 1 and c["split"] in (1, 2)
                    and c["rows"] in (1, 4)]
    monkeypatch.setattr(tune, "vector_space", vsub)
    monkeypatch.setattr(tune, "rows_space", rsub)
    monkeypatch.setattr(study, "GEMV_SIZES", {"200000": 512})
    try:
        res = study.run(sizes=(200_000,), reps=2, log=lambda *a: None)
    finally:
        ops.reset_config()
        ops.load_default_tuning()
    rep = res["sizes"]["200000"]
    assert rep["n_configs"] == len(vsub(res["cus"]))
    for op in study.OPS:
        t = rep["table2"][op]
        assert 0 < t["with_copy_cfg"] <= t["own_best"]
        assert t["tie_penalty_pct"]["min"] >= 0
    assert set(rep["copy_vs_ops"]) == set(study.OPS[1:])
    g = rep["gemv"]
    assert g["m"] == 512 and g["n_configs"] == len(rsub())
    assert 0 < g["one_row_per_group_best"] <= g["own_best"]
    md = study.markdown(res)
    assert "200000" in md
