"""Calls issued on several streams at once, and from several host threads at
once.  The binding keeps one workspace per (device, stream), the library keeps
no per-call state on the host, and every kernel is deterministic, so each
result must equal bitwise the same call issued alone on the default stream."""
from __future__ import annotations

import threading

import pytest
import torch

import workloads as W
from tests.criteria import bitwise_equal
from tests.gpu_util import host, need_gpu

pytestmark = pytest.mark.gpu


def _problems(dtype, seed):
    """Two problem sets of different sizes (so different configurations and
    workspace sizes): vectors x, y; A (m x k, row-major); v (m) for A^T v and
    w (k) for A w."""
    sets = []
    for j, (n, m, k) in enumerate([(1 << 22, 3000, 2000), (100_003, 700, 64)]):
        x = W.device_draw(n, dtype, seed, 10 + j)
        y = W.device_draw(n, dtype, seed, 20 + j)
        A = W.device_draw(m * k, dtype, seed, 30 + j).view(m, k)
        v = W.device_draw(m, dtype, seed, 40 + j)
        w = W.device_draw(k, dtype, seed, 50 + j)
        sets.append((x, y, A, v, w))
    return sets


def _calls(x, y, A, v, w):
    from paper_1409_0669_amd import ops
    return [ops.dot(x, y), ops.dot(x, y, acc="compensated"), ops.nrm2(x), ops.gemv(A, w),
            ops.gemv(A, v, trans=True), ops.gemv(A, v, trans=True, acc="compensated"), ops.axpby(0.5, x, -2.0, y)]


def _check(got, refs, what):
    assert len(got) == len(refs)
    for i, (g, r) in enumerate(zip(got, refs)):
        assert bitwise_equal(host(g), r), (what, i)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_streams_at_once(dtype):
    need_gpu()
    sets = _problems(dtype, 0)
    refs = [[host(r) for r in _calls(*p)] for p in sets]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    issued = []
    for rep in range(6):
        for i, s in enumerate(streams):
            k = (rep + i) % 2          # the two streams alternate between the problem sets
            with torch.cuda.stream(s):
                issued.append((k, _calls(*sets[k])))
    torch.cuda.synchronize()
    for j, (k, outs) in enumerate(issued):
        _check(outs, refs[k], "launch group %d, set %d" % (j, k))


def test_host_threads_with_their_own_streams():
    need_gpu()
    sets = _problems("f64", 1)
    refs = [[host(r) for r in _calls(*p)] for p in sets]
    torch.cuda.synchronize()
    results, errors = {}, []

    def worker(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                outs = [((t + r) % 2, _calls(*sets[(t + r) % 2])) for r in range(4)]
            s.synchronize()
            results[t] = outs
        except Exception as e:  # reported by the main thread
            errors.append((t, e))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads)
    assert not errors, errors
    for t, outs in results.items():
        for k, o in outs:
            _check(o, refs[k], "thread %d, set %d" % (t, k))
    assert len(results) == 4
