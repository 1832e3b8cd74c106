"""Structural checks of the compiled gfx950 code (no GPU): compiles kernel
sources to AMDGPU assembly with hipcc and checks control-flow properties that
no numerical test can establish before the kernel runs.

* No work-group barrier (s_barrier) may sit inside a loop that the compiler
  turned into an exec-masked (divergent) loop: waves of a work-group would
  execute different numbers of barriers and deadlock.
* The persistent batched kernel must draw work items in a uniform loop: the
  atomic draw sits in the outermost loop's header block with no lane-dependent
  branch around the loop, and the kernel has no barriers at all.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

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


def functions(asm: str):
    for m in re.finditer(r"^(_ZN4bwla\S+):", asm, re.M):
        end = asm.find(".Lfunc_end", m.end())
        yield m.group(1), asm[m.end():end].split("\n")


def divergent_loops_with_barrier(lines):
    """Loop headers whose loop is exec-masked (a latch that clears lanes from
    exec just before looping) and whose header-to-latch range holds s_barrier."""
    bad = []
    for h, l in enumerate(lines):
        m = re.match(r"^(\.LBB\w+):.*Loop Header", l)
        if not m:
            continue
        lab = m.group(1)
        latches = [k for k, x in enumerate(lines) if k > h and re.search(r"s_c?branch\w*\s+%s\b" % re.escape(lab), x)]
        pre = range(max(0, h - 4), h)
        masked = any("s_andn2_b64 exec, exec" in lines[q] for q in pre) or any(
            "s_andn2_b64 exec, exec" in lines[q] for k in latches for q in range(max(0, k - 4), k))
        body = lines[h:max(latches)] if latches else lines[h:h + 400]
        if any("s_andn2_b64 exec, exec" in lines[q] for q in pre):
            body = body + lines[max(0, h - 60):h]
        if masked and any("s_barrier" in b for b in body):
            bad.append(lab)
    return bad


@pytest.fixture(scope="module")
def asm_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("asm")


@pytest.mark.parametrize("ctype", ["double", "float", "__bf16"])
def test_batched_kernel_draws_work_in_a_uniform_loop(ctype, asm_dir):
    asm = compile_asm("batched", ctype, asm_dir)
    found = 0
    for name, lines in functions(asm):
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


@pytest.mark.parametrize("src", ["stream", "reduce", "gemv", "ger", "batched", "strided"])
def test_no_barrier_in_divergent_loop(src, asm_dir):
    asm = compile_asm(src, "float", asm_dir)
    hazards = [(name, bad) for name, lines in functions(asm) for bad in [divergent_loops_with_barrier(lines)] if bad]
    assert not hazards, hazards[:3]
