"""Host AddressSanitizer + UndefinedBehaviorSanitizer runs of the CPU-side code.

* The library's API layer (argument validation, overlap checks, workspace
  sizing, configuration tables, tuning-table parsing, batch-plan building),
  compiled by hipcc with the sanitizers on its host pass only and linked with
  the ordinary kernel objects, driven by the CPU tests of the C ABI, the tuner
  host logic and the batch planner.
* The oracle (oracle.c), compiled by gcc with both sanitizers, driven by its
  pinning tests.

Each runs in a child process with the matching sanitizer runtime preloaded and
BWLA_LIBRARY / ORACLE_LIBRARY naming the sanitized build; any finding ends the
child with a report (-fno-sanitize-recover=all)."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT_MARKS = ("ERROR: AddressSanitizer", "runtime error:", "SUMMARY: UndefinedBehaviorSanitizer")


def _child_env(preload: str, var: str, lib: str) -> dict:
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env[var] = lib
    # the interpreter itself is not instrumented: its allocations at exit are
    # not this code's leaks
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    return env


def _run_child(env: dict, modules) -> str:
    cmd = [sys.executable, "-m", "pytest", "-q", "-s", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *modules]
    p = subprocess.run(cmd, cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600)
    out = p.stdout
    assert p.returncode == 0, "sanitized run failed (rc %d):\n%s" % (p.returncode, out[-6000:])
    for mark in REPORT_MARKS:
        assert mark not in out, "sanitizer report:\n" + out[-6000:]
    return out


def _mapped(env: dict, code: str, path: str) -> bool:
    """True when a child that runs ``code`` under ``env`` has ``path`` mapped."""
    probe = code + "\nprint(%r in open('/proc/self/maps').read())" % os.path.realpath(path)
    p = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True, timeout=300)
    assert p.returncode == 0, p.stdout[-3000:]
    return p.stdout.strip().splitlines()[-1] == "True"


def _undefined_symbols(path: str) -> str:
    return subprocess.run(["nm", "-D", "--undefined-only", path], stdout=subprocess.PIPE, text=True,
                          check=True).stdout


def test_api_layer_under_asan_ubsan(tmp_path):
    from paper_1409_0669_amd import build as b
    lib = b.build_sanitized(str(tmp_path / "libbwla_asan.so"))
    syms = _undefined_symbols(lib)
    assert "__asan_report_load" in syms and "__ubsan_handle_" in syms  # both instrumentations are in
    env = _child_env(b.sanitizer_runtime(), "BWLA_LIBRARY", lib)
    assert _mapped(env, "from paper_1409_0669_amd import _lib", lib)
    out = _run_child(env, ["tests/test_abi.py", "tests/test_tune_host.py", "tests/test_batched.py"])
    assert " passed" in out


def test_oracle_under_asan_ubsan(tmp_path):
    import oracle
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], stdout=subprocess.PIPE, text=True,
                        check=True).stdout.strip()
    if not os.path.isabs(rt):
        pytest.skip("gcc's libasan.so is not installed")
    env = _child_env(rt, "ORACLE_LIBRARY", lib)
    assert _mapped(env, "import oracle; oracle._load()", lib)
    # control: the sanitized oracle reports a read past the end of its input
    # (a copy of 1001 entries out of a 1000-entry array)
    bad = ("import ctypes, numpy as np, oracle\n"
           "L = oracle._load(); dp = ctypes.POINTER(ctypes.c_double)\n"
           "y = np.zeros(1000); x = np.zeros(1001)\n"
           "L.o_copy(1001, y.ctypes.data_as(dp), x.ctypes.data_as(dp))\n")
    p = subprocess.run([sys.executable, "-c", bad], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True, timeout=300)
    assert p.returncode != 0 and "heap-buffer-overflow" in p.stdout, p.stdout[-3000:]
    out = _run_child(env, ["tests/test_oracle.py"])
    assert " passed" in out
