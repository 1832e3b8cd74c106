"""The paper's configuration study repeated on gfx950 (Sections 3.1-3.4).

For copy, scaled addition, inner product and norm at the paper's vector size
(two million float64 entries; Section 3) and at 2^26 entries (beyond the
256 MB Infinity Cache), every configuration of the gfx950 space
(``tune.vector_space``: work-group size 64-1024, vector width 1-16, unroll
1-4, increment global/local, work-groups per CU 1-32 or one pass) is timed.
The report gives:

* per-parameter distributions for the inner product (the paper's Figures
  1-4: increment type, vector type, local work size, number of work-groups),
  as quantiles of the fraction of peak bandwidth;
* the copy-vs-operation relation across configurations (Figure 5): rank
  correlation, and the best operation rate among configurations whose copy
  rate is within 5 % of the best copy;
* the single-configuration comparison (Table 2): every operation run with the
  copy's best configuration against its own best.  Many copy configurations
  tie within measurement noise, and which of them wins decides the penalty,
  so the report also gives the range of the penalty over every configuration
  whose copy rate is within 2 % of the best copy.

The matrix-vector product is swept over the rows-kernel space
(``tune.rows_space``: work-group size, vector width, rows per work-group,
unroll, split) at the paper's 2048 x 2048 and at 16384 x 16384.  Its Table 2
analogue runs the paper's mapping -- one work-group per row -- with the
copy's best work-group size and vector width, against the GEMV's own best;
the best of the one-row-per-work-group configurations is reported as well.

Every configuration is timed as the tuner times it (``tune.time_ms``: the
median over repetitions of a HIP-event interval around four calls launched
back to back, divided by four, each interval starting behind a 2 GiB torch
sum), so a rate is the GPU's time for the operation in a sequence of
operations, not one call's on an idle GPU nor the host's rate of issuing
calls.

Run on the GPU: ``python -m paper_1409_0669_amd.study --json OUT.json --md OUT.md``.
"""
from __future__ import annotations

import argparse
import json
import statistics
import time

import numpy as np
import torch

from . import _lib as L
from . import ops, tune

PEAK_GBS = 8000.0
OPS = ("copy", "axpby", "dot", "nrm2")
TIE_BAND = 0.02  # copy configurations this close to the best copy count as ties


def _key(c):
    return tuple(sorted(c.items()))


GEMV_SIZES = {"2000000": 2048, str(1 << 26): 16384}  # the matrix paired with each vector size


def run_gemv(m, dtype, reps, log=print):
    """{config key: GB/s} over the rows-kernel space for y = A x, A m x m."""
    space = tune.rows_space()
    w = tune.Workload("gemv", dtype, n=m, m=m, layout="row")
    t0 = time.time()
    res = tune.sweep(w, space, reps=reps)
    log("gemv %dx%d %d configs in %.0f s, best %.1f GB/s" % (m, m, len(res), time.time() - t0, res[0][2]))
    del w
    return space, {_key(c): g for c, _, g in res}


def analyse_gemv(space, rates, copy_cfg):
    keys = [k for k in (_key(c) for c in space) if k in rates]
    cfgs = [dict(k) for k in keys]
    frac = np.array([rates[k] / PEAK_GBS for k in keys])
    best = int(np.argmax(frac))
    one_row = [i for i, c in enumerate(cfgs) if c["rows"] == 1 and c["split"] == 1]
    b1 = max(one_row, key=lambda i: frac[i])
    # the paper's mapping with the copy's local size and vector width
    want = _key(dict(block=copy_cfg["block"], vec=copy_cfg["vec"], rows=1, unroll=1, split=1))
    paper = rates.get(want)
    dist = {}
    for param in ("block", "vec", "rows", "split"):
        d = {}
        for v in sorted({c[param] for c in cfgs}):
            vals = frac[np.array([c[param] == v for c in cfgs])]
            d[str(v)] = {"median": round(float(np.median(vals)), 3), "max": round(float(vals.max()), 3)}
        dist[param] = d
    return {"n_configs": len(keys), "own_best": round(float(frac[best]), 3), "own_best_config": cfgs[best],
            "one_row_per_group_best": round(float(frac[b1]), 3), "one_row_per_group_best_config": cfgs[b1],
            "copy_cfg_one_row_per_group": round(paper / PEAK_GBS, 3) if paper else None,
            "copy_cfg": {"block": copy_cfg["block"], "vec": copy_cfg["vec"]}, "distributions": dist}


def run(sizes=(2_000_000, 1 << 26), dtype=torch.float64, reps=5, log=print):
    tune._blocker = tune._Blocker()
    try:
        return _run(sizes, dtype, reps, log)
    finally:
        tune._blocker = None


def _run(sizes, dtype, reps, log):
    cus = L.lib.bwla_device_cus()
    space = tune.vector_space(cus)
    ops.reset_config()
    out = {"device": "%s, %s" % (torch.cuda.get_device_name(), torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]), "cus": cus, "configs": len(space), "sizes": {}}
    for n in sizes:
        rates = {}
        for op in OPS:
            w = tune.Workload(op, dtype, n=n)
            t0 = time.time()
            res = tune.sweep(w, space, reps=reps)
            rates[op] = {_key(c): g for c, _, g in res}
            log("n=%d %-5s %d configs in %.0f s, best %.1f GB/s" % (n, op, len(res), time.time() - t0, res[0][2]))
            del w
        out["sizes"][str(n)] = analyse(space, rates)
        m = GEMV_SIZES.get(str(n))
        if m:
            gspace, grates = run_gemv(m, dtype, reps, log)
            out["sizes"][str(n)]["gemv"] = dict(analyse_gemv(gspace, grates, out["sizes"][str(n)]["table2"]["config"]),
                                                m=m)
            ops.reset_config()
    ops.reset_config()
    return out


def analyse(space, rates):
    keys = [k for k in (_key(c) for c in space) if all(k in rates[op] for op in OPS)]
    frac = {op: np.array([rates[op][k] / PEAK_GBS for k in keys]) for op in OPS}
    cfgs = [dict(k) for k in keys]
    rep = {"n_configs": len(keys)}
    # Figures 1-4: distributions of the inner product per parameter value
    dist = {}
    for param in ("increment", "vec", "block", "grid"):
        d = {}
        for v in sorted({c[param] for c in cfgs}):
            sel = np.array([c[param] == v for c in cfgs])
            vals = frac["dot"][sel]
            d[str(v)] = {"median": round(float(np.median(vals)), 3), "p90": round(float(np.quantile(vals, 0.9)), 3),
                         "max": round(float(vals.max()), 3), "n": int(sel.sum())}
        dist[param] = d
    rep["dot_distributions"] = dist
    # Figure 5: copy against the other operations
    def ranks(a):
        r = np.empty(len(a))
        r[np.argsort(a)] = np.arange(len(a))
        return r
    best_copy = frac["copy"].max()
    near = frac["copy"] >= 0.95 * best_copy
    rel = {}
    for op in OPS[1:]:
        rho = float(np.corrcoef(ranks(frac["copy"]), ranks(frac[op]))[0, 1])
        rel[op] = {"spearman_rho": round(rho, 3), "best": round(float(frac[op].max()), 3),
                   "best_among_near_copy_best": round(float(frac[op][near].max()), 3),
                   "near_copy_best_configs": int(near.sum())}
    rep["copy_vs_ops"] = rel
    # Table 2: the copy's best configuration for every operation, and the
    # penalty over the copy's near-ties (within TIE_BAND of its best)
    i = int(np.argmax(frac["copy"]))
    ties = np.flatnonzero(frac["copy"] >= (1 - TIE_BAND) * best_copy)
    t2 = {"config": cfgs[i], "tie_band": TIE_BAND, "tie_configs": int(len(ties))}
    for op in OPS:
        own = float(frac[op].max())
        pen = 100 * (1 - frac[op][ties] / own)
        t2[op] = {"with_copy_cfg": round(float(frac[op][i]), 3), "own_best": round(own, 3),
                  "own_best_config": cfgs[int(np.argmax(frac[op]))],
                  "tie_penalty_pct": {"min": round(float(pen.min()), 1), "median": round(float(np.median(pen)), 1),
                                      "max": round(float(pen.max()), 1)}}
    rep["table2"] = t2
    return rep


def markdown(res) -> str:
    lines = ["# The paper's configuration study on %s (%d CUs)" % (res["device"], res["cus"]), "",
             "%d configurations per operation, float64, fraction of the 8 TB/s HBM peak, in GPU time (four calls "
             "per interval, each interval behind a 2 GiB torch sum)." % res["configs"], ""]
    for n, r in res["sizes"].items():
        t2 = r["table2"]
        lines += ["## n = %s" % n, "", "Single configuration chosen by the copy (Table 2 analogue): `%s`" % t2["config"], "",
                  "| operation | with the copy's config | own best | penalty | penalty over the %d copy configs within %d %% of the best copy (min / median / max) |" % (
                      t2.get("tie_configs", 0), round(100 * t2.get("tie_band", 0))),
                  "|---|---|---|---|---|"]
        for op in OPS:
            t = t2[op]
            tp = t.get("tie_penalty_pct")
            lines.append("| %s | %.3f | %.3f | %.1f %% | %s |" % (
                op, t["with_copy_cfg"], t["own_best"], 100 * (1 - t["with_copy_cfg"] / t["own_best"]),
                "%.1f / %.1f / %.1f %%" % (tp["min"], tp["median"], tp["max"]) if tp else "-"))
        lines += ["", "Copy vs the other operations across all configurations (Figure 5 analogue):", "",
                  "| operation | Spearman rho | best | best among configs within 5 % of the best copy |", "|---|---|---|---|"]
        for op, v in r["copy_vs_ops"].items():
            lines.append("| %s | %.3f | %.3f | %.3f (%d configs) |" % (op, v["spearman_rho"], v["best"],
                                                                      v["best_among_near_copy_best"], v["near_copy_best_configs"]))
        g = r.get("gemv")
        if g:
            lines += ["", "Matrix-vector product, %d x %d, over %d rows-kernel configurations:" % (g["m"], g["m"], g["n_configs"]),
                      "", "| configuration | fraction of peak |", "|---|---|",
                      "| own best `%s` | %.3f |" % (g["own_best_config"], g["own_best"]),
                      "| best with one row per work-group (the paper's mapping) `%s` | %.3f |" % (
                          g["one_row_per_group_best_config"], g["one_row_per_group_best"]),
                      "| the paper's mapping with the copy's work-group size and vector width `%s` | %s |" % (
                          g["copy_cfg"], "%.3f" % g["copy_cfg_one_row_per_group"] if g["copy_cfg_one_row_per_group"] else "-"),
                      "", "GEMV by parameter: median / max fraction of peak", ""]
            for p, d in g["distributions"].items():
                lines.append("- **%s**: " % p + "; ".join("%s: %.2f/%.2f" % (k, v["median"], v["max"]) for k, v in d.items()))
        lines += ["", "Inner product by parameter (Figures 1-4 analogue): median / 90th percentile / max fraction of peak", ""]
        for p, d in r["dot_distributions"].items():
            lines.append("- **%s**: " % p + "; ".join("%s: %.2f/%.2f/%.2f" % (k, v["median"], v["p90"], v["max"])
                                                    for k, v in d.items()))
        lines.append("")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--json", required=True)
    ap.add_argument("--md", required=True)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    res = run(reps=args.reps, log=lambda *a: print(*a, flush=True))
    with open(args.json, "w") as f:
        json.dump(res, f, indent=1)
    with open(args.md, "w") as f:
        f.write(markdown(res))
    print(markdown(res))


if __name__ == "__main__":
    main()
