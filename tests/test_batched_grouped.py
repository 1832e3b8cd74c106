"""Batched launch with one work-group per work item (the plans' default):
every problem matches the oracle; results are bitwise independent of the batch
order; graph replays equal the direct launch bitwise; a batch of one matches
the single-problem call; empty problems; the full uneven workload, every
problem; sentinel slack around the outputs stays untouched."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.batch_util import check, from_sizes, problems
from tests.criteria import TOL, bitwise_equal, check_scalar, check_vector, cond_scale, plain_reduced
from tests.gpu_util import DT, host, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _grouped(monkeypatch):
    monkeypatch.delenv("BWLA_ENABLE_UNVALIDATED_BATCH", raising=False)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_grouped_infinite_and_nan_entries(dtype):
    """Batched GEMVs and dots whose data hold +-inf or NaN: those outputs are
    the oracle's non-finite values bitwise (the compensation must not turn
    inf into NaN), the others stay within tolerance."""
    need_gpu()
    from paper_1409_0669_amd.batch import BatchPlan
    gemvs, dots = from_sizes(dtype, np.array([40, 7, 300]), np.array([500, 9000, 33]), np.array([70001, 5, 200000]),
                             seed=6)
    A0, _, _ = gemvs[0]
    A0[3, 17] = float("inf")                    # row 3 of the first GEMV
    A0[9, 2], A0[9, 400] = float("inf"), float("-inf")   # row 9: inf - inf
    gemvs[2][1][5] = float("nan")               # x of the third GEMV: every row
    dots[0][0][12345] = float("-inf")
    dots[2][1][7] = float("nan")
    for acc in ("plain", "compensated"):
        BatchPlan(gemvs, dots, acc=acc).run()
        torch.cuda.synchronize()
        for i, (A, x, y) in enumerate(gemvs):
            A64, x64 = host(A), host(x)
            ref, got = oracle.gemv(A64, x64), host(y)
            fin = np.isfinite(ref)
            assert bitwise_equal(got[~fin], ref[~fin]), (acc, "gemv", i)
            check_vector(got[fin], ref[fin], np.abs(A64[fin]) @ np.abs(x64), TOL[dtype], "gemv %d" % i,
                         plain_f32=plain_reduced(dtype, acc))
        for i, (p, q, out) in enumerate(dots):
            p64, q64 = host(p), host(q)
            check_scalar(float(out.item()), oracle.dot(p64, q64), cond_scale(dtype, acc, np.abs(p64 * q64).sum()),
                         TOL[dtype], "%s dot %d" % (acc, i))
        # the planted entries reached the outputs (signs follow the other factor)
        assert not np.isfinite(float(dots[0][2].item())) and np.isnan(float(dots[2][2].item()))
        y0 = host(gemvs[0][2])
        assert not np.isfinite(y0[3]) and not np.isfinite(y0[9])
        assert np.all(np.isnan(host(gemvs[2][2])))


@pytest.mark.parametrize("packs", [1, 4, 32])
def test_grouped_packs_per_lane(packs):
    """The packs of a GEMV row each lane of a staged tile owns (the batch
    table entry's unroll, here given to the plan): 1 puts up to 64 lanes on
    a row, 32 few; every problem against the oracle."""
    need_gpu()
    from paper_1409_0669_amd.batch import BatchPlan
    for dtype in ("f64", "f32", "bf16"):
        guards = []
        gemvs, dots = from_sizes(dtype, np.array([1, 9, 300, 64]), np.array([3, 1000, 4097, 257]),
                                 np.array([5, 70001]), seed=5, align=1, guards=guards)
        for acc in ("plain", "compensated"):
            BatchPlan(gemvs, dots, acc=acc, packs=packs, block=512).run()
            torch.cuda.synchronize()
            check(dtype, acc, gemvs, dots)
            for g in guards:
                g()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("acc", ["plain", "compensated"])
def test_grouped_matches_oracle(dtype, acc):
    need_gpu()
    from paper_1409_0669_amd.batch import BatchPlan
    gemvs, dots = problems(dtype, 40, 60, 700, 300_000)
    plan = BatchPlan(gemvs, dots, acc=acc)
    plan.run()
    torch.cuda.synchronize()
    check(dtype, acc, gemvs, dots)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_grouped_permutation_bitwise_invariant(dtype):
    need_gpu()
    from paper_1409_0669_amd.batch import BatchPlan
    gemvs, dots = problems(dtype, 30, 50, 500, 200_000, seed=1)
    p1 = BatchPlan(gemvs, dots)
    p1.run()
    torch.cuda.synchronize()
    y1 = [host(g[2]) for g in gemvs]
    d1 = [host(d[2]) for d in dots]
    for g in gemvs:
        g[2].fill_(-7.0)
    for d in dots:
        d[2].fill_(-7.0)
    rng = np.random.default_rng(9)
    pg, pd = rng.permutation(len(gemvs)), rng.permutation(len(dots))
    p2 = BatchPlan([gemvs[i] for i in pg], [dots[i] for i in pd], grid=37)
    p2.run()
    torch.cuda.synchronize()
    for i in range(len(gemvs)):
        assert bitwise_equal(host(gemvs[i][2]), y1[i])
    for i in range(len(dots)):
        assert bitwise_equal(host(dots[i][2]), d1[i])


def test_grouped_graph_replay_equals_direct():
    need_gpu()
    from paper_1409_0669_amd.batch import BatchPlan
    gemvs, dots = problems("f32", 25, 40, 600, 250_000, seed=2)
    plan = BatchPlan(gemvs, dots)
    plan.run()
    torch.cuda.synchronize()
    y_ref = [host(g[2]) for g in gemvs]
    d_ref = [host(d[2]) for d in dots]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(s)
    torch.cuda.synchronize()
    for rep in range(4):
        for g in gemvs:
            g[2].fill_(float(rep) + 0.5)   # eager work between replays
        for d in dots:
            d[2].fill_(-1.0)
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        for i in range(len(gemvs)):
            assert bitwise_equal(host(gemvs[i][2]), y_ref[i]), (rep, i)
        for i in range(len(dots)):
            assert bitwise_equal(host(dots[i][2]), d_ref[i]), (rep, i)


def test_grouped_batch_of_one_matches_single_call():
    need_gpu()
    from paper_1409_0669_amd import ops
    from paper_1409_0669_amd.batch import BatchPlan
    gemvs, dots = problems("f32", 1, 1, 3000, 900_000, seed=3)
    BatchPlan(gemvs, []).run()
    BatchPlan([], dots).run()
    A, x, y = gemvs[0]
    single = ops.gemv(A, x)
    check_vector(host(y), host(single), np.abs(host(A)) @ np.abs(host(x)), TOL["f32"])
    p, q, out = dots[0]
    single = float(ops.dot(p, q).item())
    check_scalar(float(out.item()), single, 0.0, TOL["f32"])


def test_grouped_empty_problems():
    need_gpu()
    from paper_1409_0669_amd.batch import BatchPlan
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    out = torch.full((1,), 5.0, device="cuda")
    A = torch.empty(3, 0, dtype=torch.float32, device="cuda")
    y = torch.full((3,), 5.0, device="cuda")
    BatchPlan([(A, e, y)], [(e, e, out)]).run()
    torch.cuda.synchronize()
    assert float(out.item()) == 0.0
    assert torch.all(y == 0)


def test_capture_refuses_the_default_stream():
    """A plan is recorded into a graph only on a created stream: the default
    (null) stream gives BWLA_ERR_NOT_CAPTURABLE before anything is enqueued,
    and the plan still runs afterwards."""
    need_gpu()
    from paper_1409_0669_amd import _lib as L
    from paper_1409_0669_amd.batch import BatchPlan
    p = torch.ones(1000, dtype=torch.float32, device="cuda")
    out = torch.zeros(1, device="cuda")
    plan = BatchPlan([], [(p, p, out)])
    assert L.lib.bwla_batch_capture(plan._h, None) == L.ERR_NOT_CAPTURABLE
    assert "default stream" in L.lib.bwla_last_error().decode()
    plan.run()
    torch.cuda.synchronize()
    assert float(out.item()) == 1000.0


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_grouped_full_workload_every_problem(dtype):
    """512 GEMVs with M, N log-uniform in [32, 4096] and 4096 dots with n
    log-uniform in [1e3, 1e6], Kahan/Dot2-compensated FP32 accumulation: every
    output of every problem is checked against the oracle, and a replay of
    the captured graph must equal the direct launch bitwise on every
    problem."""
    need_gpu()
    from paper_1409_0669_amd.batch import BatchPlan
    M, N, D = W.batched_sizes(0)
    guards = []
    gemvs, dots = from_sizes(dtype, M, N, D, seed=0, guards=guards)
    plan = BatchPlan(gemvs, dots, acc="compensated")
    info = plan.info()
    assert info["items"] > 0
    plan.run()
    torch.cuda.synchronize()
    check(dtype, "compensated", gemvs, dots)
    for g in guards:
        g()
    y0 = [host(g[2]) for g in gemvs]
    d0 = [host(d[2]) for d in dots]
    s = torch.cuda.Stream()
    plan.capture(s)
    plan.replay()
    torch.cuda.synchronize()
    for i, g in enumerate(gemvs):
        assert bitwise_equal(host(g[2]), y0[i]), i
    for i, d in enumerate(dots):
        assert bitwise_equal(host(d[2]), d0[i]), i


# x longer than the LDS stage of a GEMV tile: rows then use 16-byte packs when
# A's rows and x are 16-byte aligned (n a multiple of the pack width) and
# single elements otherwise; the shorter rows are staged at any alignment.
STAGE = {"f64": 3968, "f32": 7936, "bf16": 7680}  # tile_stage_elems: 32 KiB of x in V residue rows, stride padding up to 63 words


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("align", [1, 64])
@pytest.mark.parametrize("block", [64, 256, 512])
def test_grouped_every_read_mode(dtype, align, block):
    """Problem starts aligned to `align` elements: with 1, most rows, x and
    dot operands are misaligned (staged tiles and element-wise dots); with
    64, GEMVs longer than the stage take 16-byte packs when n allows."""
    need_gpu()
    from paper_1409_0669_amd.batch import BatchPlan
    cap = STAGE[dtype]
    Ms = np.array([1, 7, 33, 300, 5, 64, 3, 40])
    Ns = np.array([1, 3, 17, 1000, cap, cap + 2, cap + 8, 9001])
    Ds = np.array([0, 1, 9, 1000, 65536, 65537, 200003])
    guards = []
    gemvs, dots = from_sizes(dtype, Ms, Ns, Ds, seed=3, align=align, guards=guards)
    for acc in ("plain", "compensated"):
        plan = BatchPlan(gemvs, dots, acc=acc, block=block)
        plan.run()
        torch.cuda.synchronize()
        check(dtype, acc, gemvs, dots)
        for g in guards:  # no store past any output
            g()
        plan.close()
