"""bench.py: a one-step run prints one well-formed JSON line whose bytes per
step equal the hand count of the minimal-bytes model (copy 2ns, axpby 3ns,
dot 2ns, nrm2 ns, GEMV (mn + m + n) elements), and refuses more than one GPU."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def hand_count():
    total = 0
    for s in (4, 8):
        for n in (10 ** 5, 10 ** 6, 10 ** 7, 1 << 26):
            total += (3 + 2 + 1) * n * s
        for m in (4096, 16384):
            total += 2 * (m * m + m + m) * s
    return total


def test_bench_refuses_several_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


@pytest.mark.gpu
def test_bench_one_step_json():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup", "1",
                        "--no-extra", "--cpu-seconds", "0.5", "--settle", "0"], capture_output=True, text=True,
                       timeout=600)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["unit"] == "GB/s" and d["value"] > 0
    assert d["config"]["bytes_per_step"] == hand_count()
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and 0 < r["frac"] < 1.2
    assert r["algorithmic_bytes"] == (16384 * 16384 + 2 * 16384) * 8
    c = d["copy_ceiling"]
    assert c["gbs"] > 0 and 0 < c["dominant_frac"] < 2 and 0 < c["value_frac"] < 2
    # working sets under the 256 MiB Infinity Cache are labelled, the 2^26 vectors and 16384^2 matrices are not
    assert "axpby f32 100000" in d["cache_resident"] and "gemv f64 rowx4096" in d["cache_resident"]
    assert "axpby f64 67108864" not in d["cache_resident"] and "gemv f64 rowx16384" not in d["cache_resident"]
    # the same rows timed by the GPU (behind a blocker) as well as from the host
    assert set(d["breakdown_gpu_gbs"]) == set(d["breakdown_gbs"]) and min(d["breakdown_gpu_gbs"].values()) > 0
    # the f32 axpby at 2^26 stores a 256 MiB vector, which the cache can hold between back-to-back calls
    assert d["write_cached"] == ["axpby f32 67108864"]
    # the float64 part of the step, and its HBM-resident part, as steps of their own
    assert d["f64_step"]["bytes_per_step"] == sum((3 + 2 + 1) * n * 8 for n in (10 ** 5, 10 ** 6, 10 ** 7, 1 << 26)) \
        + sum(2 * (m * m + 2 * m) * 8 for m in (4096, 16384))
    assert set(d["f64_hbm_resident"]["operations"]) == {"axpby f64 67108864", "dot f64 67108864", "nrm2 f64 67108864",
                                                        "gemv f64 rowx16384", "gemv f64 colx16384"}
    assert d["small_fp64_set"]["cache_resident"] and d["small_fp64_set"]["dot f64 n=2^20"]["GB/s"] > 0
    # the CPU leg: the oracle over the whole step, the naive loops, the host, every step row's error
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["cores"] == 1 and cpu["value"] > 0
    assert cpu["naive_fp64"]["cores"] >= 1 and cpu["naive_fp64"]["value"] > 0
    assert cpu["host"]["os_cpu_count"] >= 1 and cpu["host"]["affinity_cpus"] >= 1
    acc = d["accuracy"]
    assert set(acc["step"]) == set(d["breakdown_gbs"])
    assert all(r["within_tol"] for r in acc["step"].values()), acc["step"]
    assert acc["step"]["axpby f64 67108864"]["max_ulp"] == 0
    assert acc["step"]["dot f64 67108864"]["rel"] <= 1e-12 and acc["all_within_tol"]


def test_error_measures():
    """The accuracy report's measures on values with known distances: ULPs in
    each storage format (across zero and for negative values too), the
    relative and condition-scaled bounds, and the two GEMV measures."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    one = np.array([1.0])
    assert bench.err_elementwise(one, one, "f64") == {"max_ulp": 0, "within_tol": True}
    assert bench.err_elementwise(np.array([1.0 + 2.0 ** -52]), one, "f64")["max_ulp"] == 1
    assert bench.err_elementwise(np.array([1.0 + 2.0 ** -50]), one, "f64")["max_ulp"] == 4
    assert bench.err_elementwise(np.array([-1.0]), np.array([-1.0 - 2.0 ** -52]), "f64")["max_ulp"] == 1
    tiny = 5e-324  # the smallest subnormal: -tiny and +tiny are 2 ULPs apart (through +-0)
    assert bench.err_elementwise(np.array([-tiny]), np.array([tiny]), "f64")["max_ulp"] == 2
    assert bench.err_elementwise(np.array([1.0 + 2.0 ** -23]), one, "f32")["max_ulp"] == 1
    assert bench.err_elementwise(np.array([1.0 + 2.0 ** -7]), one, "bf16")["max_ulp"] == 1
    assert bench.err_elementwise(np.array([2.0]), one, "bf16")["max_ulp"] == 128
    e = (1.0 + 2e-12) - 1.0  # the difference of the two doubles, about 2e-12
    r = bench.err_scalar(1.0 + 2e-12, 1.0, "f64", 100.0)
    assert not r["within_tol"] and r["rel"] == e and r["cond"] == e / 100.0  # f64 is judged on |ref| alone
    assert bench.err_scalar(1.0 + 5e-4, 1.0, "f32", 100.0, cond=True)["within_tol"]   # 5e-4 <= 1e-5 * 100
    assert not bench.err_scalar(1.0 + 5e-4, 1.0, "f32", 100.0)["within_tol"]
    g = bench.err_gemv(np.array([1.0, 3e-13]), np.array([1.0, 0.0]), np.array([1.0, 1.0]), "f64")
    assert g["componentwise"] == 3e-13 and g["normwise"] == 3e-13 and g["within_tol"]
    g = bench.err_gemv(np.array([1.0, 0.0]), np.array([1.0, 2e-12]), np.array([1.0, 1.0]), "f64")
    assert not g["within_tol"]


def test_write_cached_rule():
    """A row is flagged when its stores are at least 5 % of its bytes and fit
    the 256 MiB Infinity Cache."""
    sys.path.insert(0, ROOT)
    import bench
    mib = 1 << 20
    assert bench._write_cached(768 * mib, 256 * mib)
    assert not bench._write_cached(1536 * mib, 512 * mib)
    assert not bench._write_cached(2048 * mib, 64 * 1024)  # a GEMV's output vector
    assert not bench._write_cached(1024 * mib, 0)
    assert bench._step_written(("axpby", "f32", 1 << 26)) == 256 * mib
    assert bench._step_written(("dot", "f64", 1 << 26)) == 0
    assert bench._step_written(("gemv", "f64", "row", 16384)) == 0
