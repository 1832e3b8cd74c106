"""Structural checks of the compiled gfx950 code (no GPU): compiles kernel
sources to AMDGPU assembly with hipcc and checks control-flow properties that
no numerical test can establish before the kernel runs.

* No work-group barrier (s_barrier) may sit inside a loop that the compiler
  turned into an exec-masked (divergent) loop: waves of a work-group would
  execute different numbers of barriers and deadlock.
* The persistent batched kernel must draw work items in a uniform loop: the
  atomic draw sits in the outermost loop's header block with no lane-dependent
  branch around the loop, and the kernel has no barriers at all.
* Every streaming, reduction and GEMV instantiation that fits its registers
  keeps (at least three quarters of) the loads of an unrolled trip in flight
  at once -- the bytes in flight per wave are what the unroll and
  vector-width axes buy; the machine scheduler may not sink part of them into
  the arithmetic.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1409_0669_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


def compile_asm(src: str, ctype: str, out_dir) -> str:
    out = os.path.join(str(out_dir), "%s_%s.s" % (src, ctype.strip("_")))
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-DBWLA_T=%s" % ctype, "-DBWLA_T_IS_F64=1", "--offload-device-only", "-S",
           os.path.join(CSRC, src + ".hip"), "-o", out]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return open(out).read()


def functions(asm: str, prefix: str = "_ZN4bwla"):
    for m in re.finditer(r"^(%s\S+):" % prefix, asm, re.M):
        end = asm.find(".Lfunc_end", m.end())
        yield m.group(1), asm[m.end():end].split("\n")


def loop_structure(lines):
    """Blocks and loops from the compiler's block annotations.  Returns
    (blocks, loops): blocks is a list of (start, end, innermost loop header
    or None); loops maps a header to the list of its enclosing headers.  A
    header's label line (and its comment continuation lines) names its
    parent loops ("Parent Loop BBx Depth=k") and itself ("Loop Header"); any
    other block of a loop says "in Loop: Header=BBx"."""
    starts = [i for i, l in enumerate(lines) if re.match(r"^(\.LBB\w+:|; %bb\.\d+:)", l)]
    blocks, loops = [], {}
    for b, i in enumerate(starts):
        end = starts[b + 1] if b + 1 < len(starts) else len(lines)
        note = lines[i]
        k = i + 1
        while k < end and re.match(r"^\s+;", lines[k]):
            note += lines[k]
            k += 1
        m = re.match(r"^\.L(BB\w+):", lines[i])
        if "Loop Header" in note and m:
            loops[m.group(1)] = re.findall(r"Parent Loop (BB\w+)", note)
            blocks.append((i, end, m.group(1)))
        else:
            h = re.search(r"in Loop: Header=(BB\w+)", note)
            blocks.append((i, end, h.group(1) if h else None))
    return blocks, loops


def divergent_loops_with_barrier(lines):
    """Headers of exec-masked loops (lanes leave the loop one by one: the
    loop's own blocks clear exiting lanes with s_andn2_b64 exec, exec, ...)
    that hold an s_barrier, directly or in a loop nested inside them."""
    blocks, loops = loop_structure(lines)
    masked = set()
    for start, end, h in blocks:
        if h and any("s_andn2_b64 exec, exec" in l for l in lines[start:end]):
            masked.add(h)
    bad = []
    for start, end, h in blocks:
        if h is None or not any("s_barrier" in l for l in lines[start:end]):
            continue
        for enclosing in [h] + loops.get(h, []):
            if enclosing in masked and enclosing not in bad:
                bad.append(enclosing)
    return bad


@pytest.fixture(scope="module")
def asm_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("asm")


# every (source, storage type) the checks below read, compiled in parallel once
SOURCES = [(src, "float") for src in ("stream", "reduce", "gemv", "ger", "batched", "strided")] + \
          [(src, t) for src in ("stream", "reduce", "gemv", "batched") for t in ("double", "__bf16")]


@pytest.fixture(scope="module")
def asm(asm_dir):
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        texts = list(ex.map(lambda st: compile_asm(st[0], st[1], asm_dir), SOURCES))
    return dict(zip(SOURCES, texts))


@pytest.mark.parametrize("ctype", ["double", "float", "__bf16"])
def test_batched_kernel_draws_work_in_a_uniform_loop(ctype, asm):
    found = 0
    for name, lines in functions(asm[("batched", ctype)]):
        if "k_batched" not in name:
            continue
        found += 1
        text = "\n".join(lines)
        assert "s_barrier" not in text, name
        # the outermost loop header and the block that follows it
        h = next(k for k, l in enumerate(lines) if "Loop Header: Depth=1" in l)
        head_block = []
        for l in lines[h + 1:]:
            if re.match(r"^\.LBB\w+:.*Depth=1", l) and "Inner Loop" not in l and "Parent Loop" not in l:
                break
            head_block.append(l)
            if "s_cbranch" in l and "LBB" in l and "vcc" in l:
                break
        assert any("global_atomic_add" in l for l in head_block), name
        # the outermost loop is not exec-masked: no latch rewrites exec
        lab = re.match(r"^(\.LBB\w+):", lines[h]).group(1)
        latches = [k for k, l in enumerate(lines) if re.search(r"s_c?branch\w*\s+%s\b" % re.escape(lab), l)]
        for k in latches:
            assert not any("s_andn2_b64 exec, exec" in lines[q] for q in range(max(0, k - 4), k)), name
        assert not any("s_andn2_b64 exec, exec" in lines[q] for q in range(max(0, h - 4), h)), name
    assert found == 4


def test_detector_on_fixture(asm_dir):
    """The checker flags a barrier inside a lane-dependent loop and passes
    one placed after such a loop (host-compiled fixture, never launched)."""
    out = os.path.join(str(asm_dir), "fixture.s")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "--offload-device-only", "-S",
                    os.path.join(ROOT, "tests", "isa_fixtures", "barrier_loop.hip"), "-o", out],
                   check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    found = dict((name, divergent_loops_with_barrier(lines)) for name, lines in functions(open(out).read(), "_Z"))
    bad = [v for k, v in found.items() if "barrier_in_lane_dependent_loop" in k]
    good = [v for k, v in found.items() if "barrier_after_lane_dependent_loop" in k]
    assert len(bad) == 1 and bad[0], found
    assert len(good) == 1 and not good[0], found


@pytest.mark.parametrize("src", ["stream", "reduce", "gemv", "ger", "batched", "strided"])
def test_no_barrier_in_divergent_loop(src, asm):
    hazards = [(name, bad) for name, lines in functions(asm[(src, "float")])
               for bad in [divergent_loops_with_barrier(lines)] if bad]
    assert not hazards, hazards[:3]


def loads_in_flight(lines):
    """Most vector-memory loads outstanding at once inside any basic block
    (each block starts from none; s_waitcnt vmcnt(k) leaves at most k)."""
    best = cur = 0
    for l in lines:
        t = l.strip()
        if re.match(r"^(\.LBB\w+:|; %bb\.\d+:)", t):
            cur = 0
        elif re.match(r"(global|buffer|flat)_load", t):
            cur += 1
            best = max(best, cur)
        else:
            m = re.match(r"s_waitcnt\s.*vmcnt\((\d+)\)", t)
            if m:
                cur = min(cur, int(m.group(1)))
    return best


KERNEL = re.compile(r"_ZN4bwla\d+(k_\w+?)I(?:d|f|DF16b)?((?:L[ib]\d+E)+)E")
ELEM = {"double": 8, "float": 4, "__bf16": 2}


def trip_loads(kernel, args, es):
    """Loads one unrolled trip issues, from the template arguments (a pack of
    V elements is max(1, V * es / 16) 16-byte loads)."""
    lp = lambda v: max(1, v * es // 16)
    if kernel in ("k_copy", "k_scal"):
        return args[1] * lp(args[0])
    if kernel == "k_axpby":
        return 2 * args[1] * lp(args[0])
    if kernel == "k_cg":
        return 4 * args[1] * lp(args[0])
    if kernel == "k_dot":          # <V, U, COMP, MODE>: two streams for the inner product
        return args[1] * lp(args[0]) * (2 if args[3] == 0 else 1)
    if kernel == "k_gemv_rows":    # <V, R, U, COMP>: R lines of A and the x pack per trip
        return args[2] * (args[1] + 1) * lp(args[0])
    if kernel == "k_gemv_cols":    # <V, U, COMP>: U lines
        return args[1] * lp(args[0])
    if kernel == "k_combine_lines":   # <COMP, B>: a batch of B 16-byte partials
        return args[1]
    if kernel == "k_combine_scalar":  # <COMP>: a batch of eight 16-byte partials
        return 8
    return None


@pytest.mark.parametrize("src", ["stream", "reduce", "gemv"])
@pytest.mark.parametrize("ctype", ["double", "float", "__bf16"])
def test_unrolled_trips_keep_every_load_in_flight(src, ctype, asm):
    text = asm[(src, ctype)]
    spills = {m.group(1): int(re.search(r"\.vgpr_spill_count:\s+(\d+)", m.group(2)).group(1))
              for m in re.finditer(r"\.name:\s+(\S+)\n(.*?)(?=\n  - \.|\Z)", text, re.S)
              if re.search(r"\.vgpr_spill_count:", m.group(2))}
    checked, short = 0, []
    for name, lines in functions(text):
        m = KERNEL.match(name)
        if not m or spills.get(name, 0):
            continue  # not an unrolled streaming kernel, or it cannot hold a trip in registers
        args = [int(v) for v in re.findall(r"L[ib](\d+)E", m.group(2))]
        want = trip_loads(m.group(1), args, ELEM[ctype])
        if want is None:
            continue
        checked += 1
        got = loads_in_flight(lines)
        # at least three quarters: the instruction selector may still place a
        # conversion that consumes the first loads ahead of the last ones
        # (bf16 pairs of the four-stream update), which costs little; a trip
        # cut to a few loads in flight costs half the bandwidth
        if 4 * got < 3 * want:
            short.append((m.group(1), args, got, want))
    assert checked >= 20, checked
    assert not short, short[:5]
