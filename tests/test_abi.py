"""The C-ABI library: it loads, exports every symbol the header declares, and
rejects invalid arguments with the documented status before touching the GPU.
These tests make no compute call and run without a GPU."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1409_0669_amd import _lib
    return _lib


def header_functions():
    text = open(os.path.join(ROOT, "include", "bwla.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bwla_\w+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L.lib, n), n
    # and the binding declares a signature for each of them
    assert set(names) == set(L.SIGNATURES), set(names) ^ set(L.SIGNATURES)


def test_abi_version_and_strings(L):
    assert L.lib.bwla_abi_version() == L.ABI_VERSION == 4
    for st, name in [(0, b"ok"), (1, b"invalid argument"), (3, b"workspace too small"), (4, b"HIP error")]:
        assert L.lib.bwla_status_string(st) == name


FAKE = 1 << 40  # an address that is never dereferenced: validation fails first


def st(L, r):
    return r, L.lib.bwla_last_error().decode()


def test_unknown_enum_values_are_rejected(L):
    """Every entry point rejects a storage type, accumulation mode or output
    type it does not know with the documented status, before any table
    lookup (the host-sanitizer run of this module checks that no lookup reads
    outside its table)."""
    lib = L.lib
    G = 1 << 30
    x, y, z, out, ws, A = FAKE, FAKE + G, FAKE + 2 * G, FAKE + 3 * G, FAKE + 4 * G, FAKE + 8 * G
    sz = ctypes.c_size_t(0)
    cfg = L.Config()
    calls = {
        "copy": lambda t, a, o: lib.bwla_copy(t, 10, y, x, None),
        "axpby": lambda t, a, o: lib.bwla_axpby(t, 10, 1.0, None, y, 1.0, None, z, x, None),
        "dot": lambda t, a, o: lib.bwla_dot(t, a, 10, x, y, o, out, ws, G, None),
        "nrm2": lambda t, a, o: lib.bwla_nrm2(t, a, 10, x, o, out, ws, G, None),
        "dot_noalloc": lambda t, a, o: lib.bwla_dot_noalloc(t, a, 10, x, y, o, out, None),
        "dot_strided": lambda t, a, o: lib.bwla_dot_strided(t, a, 10, x, 2, y, 3, o, out, ws, G, None),
        "nrm2_strided": lambda t, a, o: lib.bwla_nrm2_strided(t, a, 10, x, 2, o, out, ws, G, None),
        "asum": lambda t, a, o: lib.bwla_asum(t, a, 10, x, 2, o, out, ws, G, None),
        "copy_strided": lambda t, a, o: lib.bwla_copy_strided(t, 10, y, 2, x, 3, None),
        "axpby_strided": lambda t, a, o: lib.bwla_axpby_strided(t, 10, 1.0, None, y, 2, 1.0, None, z, 2, x, 3,
                                                                None),
        "scal": lambda t, a, o: lib.bwla_scal(t, 10, 2.0, None, x, 2, None),
        "scal_to": lambda t, a, o: lib.bwla_scal_to(t, 10, 2.0, None, y, x, None),
        "gemv": lambda t, a, o: lib.bwla_gemv(t, a, 0, 0, 8, 8, A, 8, x, o, y, ws, G, None),
        "gemv_dot": lambda t, a, o: lib.bwla_gemv_dot(t, a, 0, 0, 8, 8, A, 8, x, y, z, o, out, ws, G, None),
        "gemv_dot_ws": lambda t, a, o: lib.bwla_gemv_dot_workspace_size(t, 0, 0, 8, 8, ctypes.byref(sz)),
        "gemv_ex": lambda t, a, o: lib.bwla_gemv_ex(t, a, 0, 0, 8, 8, 1.0, A, 8, x, 2, 0.5, o, y, 2, ws, G, None),
        "gemv_ex_ws": lambda t, a, o: lib.bwla_gemv_ex_workspace_size(t, o, 0, 0, 8, 8, ctypes.byref(sz)),
        "ger": lambda t, a, o: lib.bwla_ger(t, 0, 8, 8, x, y, A, 8, None),
        "cg_update": lambda t, a, o: lib.bwla_cg_update(t, a, 10, 1.0, None, x, y, z, A, o, out, ws, G, None),
        "workspace_size": lambda t, a, o: lib.bwla_workspace_size(L.OP_DOT, t, a, 0, 0, 1, 1000, ctypes.byref(sz)),
        "get_config": lambda t, a, o: lib.bwla_get_config(L.OP_DOT, t, a, 1, 1000, ctypes.byref(cfg)),
    }
    with_acc = {"dot", "nrm2", "dot_noalloc", "dot_strided", "nrm2_strided", "asum", "gemv", "gemv_dot",
                "gemv_ex", "cg_update", "workspace_size", "get_config"}
    with_out = {"dot", "nrm2", "dot_noalloc", "dot_strided", "nrm2_strided", "asum", "gemv", "gemv_dot",
                "gemv_ex", "gemv_ex_ws", "cg_update"}
    for name, call in calls.items():
        for bad in (3, 7, 99, -1, 2 ** 31 - 1):
            assert call(bad, 0, 0) == L.ERR_UNSUPPORTED, (name, "dtype", bad)
            if name in with_acc:
                assert call(0, bad, 0) == L.ERR_UNSUPPORTED, (name, "acc", bad)
            if name in with_out:
                assert call(0, 0, bad) in (L.ERR_UNSUPPORTED, L.ERR_INVALID_ARG), (name, "out type", bad)
    for bad in (-2, L.OP_COUNT, 99):
        assert lib.bwla_get_config(bad, 0, 0, 1, 1000, ctypes.byref(cfg)) == L.ERR_INVALID_ARG
        assert lib.bwla_set_config(bad, 0, 0, 1, None) == L.ERR_INVALID_ARG
    for bad in (3, 7, -1):
        assert lib.bwla_set_config(L.OP_DOT, bad, 0, 1, None) == L.ERR_UNSUPPORTED


def test_unroll_limits(L):
    """unroll takes 1..32 (powers of two); each operation keeps to what its
    kernels have: the streaming operations 4, the reductions 8, the cols
    GEMV 32 while those lines hold at most 128 bytes of A per lane."""
    import torch
    from paper_1409_0669_amd import ops
    lib = L.lib
    for bad in (3, 64, -1):
        assert lib.bwla_set_config(L.OP_DOT, 0, -1, -1, ctypes.byref(L.Config(unroll=bad))) == L.ERR_INVALID_ARG
    try:
        for dt, vec, want in ((torch.float32, 1, 32), (torch.float32, 2, 16), (torch.float32, 4, 8),
                              (torch.float64, 1, 16), (torch.float64, 2, 8), (torch.bfloat16, 2, 32),
                              (torch.bfloat16, 8, 8)):
            ops.set_config(L.OP_GEMV_COLS, dt, -1, block=1024, vec=vec, unroll=32)
            assert ops.get_config(L.OP_GEMV_COLS, dt, 4096, 4096)["unroll"] == want, (dt, vec)
        ops.set_config(L.OP_DOT, torch.float32, -1, unroll=32)
        assert ops.get_config(L.OP_DOT, torch.float32, 0, 1 << 20)["unroll"] == 8
        ops.set_config(L.OP_AXPBY, torch.float32, -1, unroll=16)
        assert ops.get_config(L.OP_AXPBY, torch.float32, 0, 1 << 20)["unroll"] == 4
    finally:
        ops.reset_config()


def test_batch_configuration_from_the_table(L):
    """Batch plans take their work-group size and packs per lane from the
    BWLA_OP_BATCH entry of the plan's size class (by algorithmic bytes);
    defaults 256 threads and 16 packs; work-groups are capped at 512."""
    import torch
    from paper_1409_0669_amd import ops
    try:
        ops.reset_config()
        got = ops.get_config(L.OP_BATCH, torch.float32, 0, 3 << 30)
        assert (got["block"], got["unroll"]) == (256, 16)
        ops.set_config(L.OP_BATCH, torch.float32, 4, acc="compensated", block=512, unroll=8)
        got = ops.get_config(L.OP_BATCH, torch.float32, 0, 3 << 30, acc="compensated")
        assert (got["block"], got["unroll"]) == (512, 8)
        assert ops.get_config(L.OP_BATCH, torch.float32, 0, 3 << 30)["unroll"] == 16      # the other mode
        assert ops.get_config(L.OP_BATCH, torch.float32, 0, 1 << 20, acc="compensated")["unroll"] == 16  # class
        ops.set_config(L.OP_BATCH, torch.bfloat16, -1, block=1024)
        assert ops.get_config(L.OP_BATCH, torch.bfloat16, 0, 3 << 30)["block"] == 512
    finally:
        ops.reset_config()


def test_vector_validation(L):
    lib = L.lib
    assert lib.bwla_copy(0, -1, FAKE, FAKE + 4096, None) == L.ERR_INVALID_ARG
    assert lib.bwla_copy(7, 10, FAKE, FAKE + 4096, None) == L.ERR_UNSUPPORTED
    assert lib.bwla_copy(0, 10, None, FAKE, None) == L.ERR_INVALID_ARG
    assert lib.bwla_copy(0, 0, None, None, None) == L.OK          # empty: nothing to do
    # partial overlap x = y + 1 element
    assert lib.bwla_copy(0, 10, FAKE, FAKE + 8, None) == L.ERR_INVALID_ARG
    assert lib.bwla_axpby(0, 10, 1.0, None, FAKE, 1.0, None, FAKE + 8000, FAKE + 8, None) == L.ERR_INVALID_ARG
    assert "overlap" in lib.bwla_last_error().decode()
    assert lib.bwla_axpby(0, -5, 1.0, None, FAKE, 1.0, None, FAKE, FAKE, None) == L.ERR_INVALID_ARG
    assert lib.bwla_axpby(0, 5, 1.0, None, None, 1.0, None, FAKE, FAKE, None) == L.ERR_INVALID_ARG
    # device scalar inside the output
    assert lib.bwla_axpby(0, 10, 1.0, FAKE + 16, FAKE + 4096, 1.0, None, FAKE + 8192, FAKE, None) == L.ERR_INVALID_ARG


def test_reduction_validation(L):
    lib = L.lib
    out = FAKE + (1 << 20)
    assert lib.bwla_dot(0, 0, -1, FAKE, FAKE, 0, out, None, 0, None) == L.ERR_INVALID_ARG
    assert lib.bwla_dot(0, 5, 10, FAKE, FAKE, 0, out, None, 0, None) == L.ERR_UNSUPPORTED
    assert lib.bwla_dot(0, 0, 10, FAKE, FAKE, 1, out, None, 0, None) == L.ERR_UNSUPPORTED  # f64 -> f32 out
    assert lib.bwla_dot(1, 0, 10, FAKE, FAKE, 2, out, None, 0, None) == L.ERR_UNSUPPORTED  # bf16 out
    assert lib.bwla_dot(0, 0, 10, FAKE, FAKE, 0, None, None, 0, None) == L.ERR_INVALID_ARG
    # a long dot needs a workspace
    assert lib.bwla_dot(0, 0, 1 << 24, FAKE, FAKE + (1 << 28), 0, out, None, 0, None) == L.ERR_WORKSPACE
    assert lib.bwla_dot(0, 0, 1 << 24, FAKE, FAKE + (1 << 28), 0, out, FAKE + (1 << 30), 100, None) == L.ERR_WORKSPACE
    # output inside an input
    assert lib.bwla_dot(0, 0, 100, FAKE, FAKE + 4096, 0, FAKE + 64, FAKE + (1 << 30), 1 << 20, None) == L.ERR_INVALID_ARG
    assert lib.bwla_nrm2(0, 0, -3, FAKE, 0, out, None, 0, None) == L.ERR_INVALID_ARG
    assert lib.bwla_cg_update(0, 0, 10, 1.0, None, FAKE, FAKE, FAKE, FAKE, 0, out, FAKE + (1 << 30), 1 << 20,
                              None) == L.ERR_INVALID_ARG  # x overlaps r


def test_gemv_validation(L):
    lib = L.lib
    y = FAKE + (1 << 34)
    x = FAKE + (1 << 33)
    A = FAKE
    assert lib.bwla_gemv(0, 0, 0, 0, 10, 20, A, 19, x, 0, y, None, 0, None) == L.ERR_INVALID_ARG  # lda < n
    assert lib.bwla_gemv(0, 0, 1, 0, 10, 20, A, 9, x, 0, y, None, 0, None) == L.ERR_INVALID_ARG   # col: lda < m
    assert lib.bwla_gemv(0, 0, 2, 0, 10, 20, A, 20, x, 0, y, None, 0, None) == L.ERR_INVALID_ARG  # layout
    assert lib.bwla_gemv(0, 0, 0, 2, 10, 20, A, 20, x, 0, y, None, 0, None) == L.ERR_INVALID_ARG  # trans
    assert lib.bwla_gemv(0, 0, 0, 0, -1, 20, A, 20, x, 0, y, None, 0, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv(0, 0, 0, 0, 10, 20, None, 20, x, 0, y, None, 0, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv(0, 0, 0, 0, 10, 20, A, 20, x, 0, A + 80, None, 0, None) == L.ERR_INVALID_ARG  # y in A
    assert lib.bwla_gemv(0, 0, 0, 0, 0, 20, A, 20, x, 0, None, None, 0, None) == L.OK  # no outputs
    assert lib.bwla_gemv(2, 0, 0, 0, 10, 20, A, 20, x, 2, y, None, 0, None) == L.ERR_UNSUPPORTED  # bf16 out
    assert lib.bwla_ger(0, 0, 10, 20, x, x + 800, A, 19, None) == L.ERR_INVALID_ARG
    assert lib.bwla_ger(0, 0, 10, 20, A + 8, x, A, 20, None) == L.ERR_INVALID_ARG  # u inside A
    assert lib.bwla_ger(0, 0, 0, 20, None, None, None, 20, None) == L.OK


def test_workspace_sizes(L):
    lib = L.lib
    b = ctypes.c_size_t()
    assert lib.bwla_workspace_size(L.OP_DOT, 0, 0, 0, 0, 0, 1 << 26, ctypes.byref(b)) == L.OK
    assert b.value > 0
    assert lib.bwla_workspace_size(L.OP_GEMV_ROWS, 0, 0, 1, 0, 16384, 16384, ctypes.byref(b)) == L.OK
    col = b.value
    assert col > 0          # column-major y = A x splits across lines
    assert lib.bwla_workspace_size(L.OP_GEMV_ROWS, 0, 0, 0, 0, 16384, 16384, ctypes.byref(b)) == L.OK
    assert lib.bwla_workspace_size(L.OP_DOT, 0, 0, 0, 0, -1, 5, ctypes.byref(b)) == L.ERR_INVALID_ARG


def test_config_table(L):
    lib = L.lib
    c = L.Config(block=512, vec=4, unroll=2, grid=1024, increment=1, rows=0, split=0)
    assert lib.bwla_set_config(L.OP_AXPBY, 1, -1, -1, ctypes.byref(c)) == L.OK
    got = L.Config()
    assert lib.bwla_get_config(L.OP_AXPBY, 1, 0, 0, 1000, ctypes.byref(got)) == L.OK
    assert (got.block, got.vec, got.unroll, got.grid, got.increment) == (512, 4, 2, 1024, 1)
    assert lib.bwla_set_config(L.OP_AXPBY, 1, -1, -1, None) == L.OK
    assert lib.bwla_get_config(L.OP_AXPBY, 1, 0, 0, 1000, ctypes.byref(got)) == L.OK
    assert (got.block, got.vec) == (256, 4)
    bad = L.Config(block=100)
    assert lib.bwla_set_config(L.OP_COPY, 0, -1, 0, ctypes.byref(bad)) == L.ERR_INVALID_ARG
    bad = L.Config(vec=3)
    assert lib.bwla_set_config(L.OP_COPY, 0, -1, 0, ctypes.byref(bad)) == L.ERR_INVALID_ARG
    assert lib.bwla_set_config(99, 0, -1, 0, None) == L.ERR_INVALID_ARG
    assert lib.bwla_set_config(L.OP_DOT, 0, 2, 0, None) == L.ERR_INVALID_ARG      # no such mode
    assert lib.bwla_get_config(L.OP_DOT, 0, 2, 0, 10, ctypes.byref(got)) == L.ERR_UNSUPPORTED
    # eight packs in flight: kept for the reductions, four for everything else
    eight = L.Config(unroll=8)
    for op, want in ((L.OP_DOT, 8), (L.OP_NRM2, 8), (L.OP_COPY, 4), (L.OP_AXPBY, 4), (L.OP_CG, 4),
                     (L.OP_GEMV_COLS, 8), (L.OP_GEMV_ROWS, 1)):
        assert lib.bwla_set_config(op, 0, -1, -1, ctypes.byref(eight)) == L.OK
        assert lib.bwla_get_config(op, 0, 0, 1024, 1 << 20, ctypes.byref(got)) == L.OK
        assert got.unroll == want, (op, got.unroll)
        assert lib.bwla_set_config(op, 0, -1, -1, None) == L.OK
    assert lib.bwla_set_config(L.OP_DOT, 0, -1, -1, ctypes.byref(L.Config(unroll=3))) == L.ERR_INVALID_ARG


def test_config_table_keeps_the_accumulation_modes_apart(L):
    """The reducing operations have one entry per accumulation mode; the
    elementwise ones read their plain entry whatever mode a caller names."""
    lib = L.lib
    got = L.Config()
    plain, comp = L.Config(block=1024, vec=2, unroll=4, grid=256), L.Config(block=256, vec=1, unroll=2, grid=512)
    try:
        for op in (L.OP_DOT, L.OP_NRM2, L.OP_CG):
            assert lib.bwla_set_config(op, 1, L.ACC_PLAIN, -1, ctypes.byref(plain)) == L.OK
            assert lib.bwla_set_config(op, 1, L.ACC_COMPENSATED, -1, ctypes.byref(comp)) == L.OK
            for acc, want in ((L.ACC_PLAIN, plain), (L.ACC_COMPENSATED, comp)):
                assert lib.bwla_get_config(op, 1, acc, 0, 1 << 22, ctypes.byref(got)) == L.OK
                assert (got.block, got.vec, got.unroll, got.grid) == (want.block, want.vec, want.unroll,
                                                                       want.grid), (op, acc)
        rows_p, rows_c = L.Config(block=512, vec=4, rows=4, split=1), L.Config(block=256, vec=4, rows=2, split=2)
        assert lib.bwla_set_config(L.OP_GEMV_ROWS, 1, L.ACC_PLAIN, -1, ctypes.byref(rows_p)) == L.OK
        assert lib.bwla_set_config(L.OP_GEMV_ROWS, 1, L.ACC_COMPENSATED, -1, ctypes.byref(rows_c)) == L.OK
        lib.bwla_get_config(L.OP_GEMV_ROWS, 1, L.ACC_PLAIN, 4096, 4096, ctypes.byref(got))
        assert (got.block, got.rows, got.split) == (512, 4, 1)
        lib.bwla_get_config(L.OP_GEMV_ROWS, 1, L.ACC_COMPENSATED, 4096, 4096, ctypes.byref(got))
        assert (got.block, got.rows, got.split) == (256, 2, 2)
        # the workspace size covers both modes: a compensated entry with more
        # work-groups raises the size asked for in plain mode too
        b_small, b_big = ctypes.c_size_t(), ctypes.c_size_t()
        assert lib.bwla_set_config(L.OP_DOT, 1, -1, -1, ctypes.byref(L.Config(grid=256))) == L.OK
        lib.bwla_workspace_size(L.OP_DOT, 1, L.ACC_PLAIN, 0, 0, 0, 1 << 22, ctypes.byref(b_small))
        assert lib.bwla_set_config(L.OP_DOT, 1, L.ACC_COMPENSATED, -1, ctypes.byref(L.Config(grid=4096))) == L.OK
        lib.bwla_workspace_size(L.OP_DOT, 1, L.ACC_PLAIN, 0, 0, 0, 1 << 22, ctypes.byref(b_big))
        assert b_big.value >= 4096 * 16 > b_small.value
        # elementwise operations: one entry, whichever mode is named
        assert lib.bwla_set_config(L.OP_AXPBY, 1, L.ACC_COMPENSATED, -1, ctypes.byref(comp)) == L.OK
        lib.bwla_get_config(L.OP_AXPBY, 1, L.ACC_COMPENSATED, 0, 1 << 22, ctypes.byref(got))
        assert got.block == 256 and got.grid != 512   # the plain (default) entry
        assert lib.bwla_workspace_size(L.OP_DOT, 1, 2, 0, 0, 0, 10, ctypes.byref(b_big)) == L.ERR_UNSUPPORTED
    finally:
        for op in range(L.OP_COUNT):
            lib.bwla_set_config(op, 1, -1, -1, None)


def test_load_tuning(L, tmp_path):
    lib = L.lib
    p = tmp_path / "t.txt"
    p.write_text("# op dtype acc class block vec unroll grid inc rows split\n"
                 "1 0 -1 -1 512 2 2 0 0 0 0   # axpby f64\n\n"
                 "3 1 -1 4 256 4 1 0 0 8 2\n"   # class 4: at least 1 GiB
                 "2 1 0 -1 1024 4 4 256 0 0 0\n"
                 "2 1 1 -1 256 4 2 512 1 0 0\n")
    assert lib.bwla_load_tuning(str(p).encode()) == L.OK
    got = L.Config()
    lib.bwla_get_config(L.OP_AXPBY, 0, 0, 0, 1 << 20, ctypes.byref(got))
    assert (got.block, got.vec, got.unroll) == (512, 2, 2)
    for acc in (0, 1):
        lib.bwla_get_config(L.OP_GEMV_ROWS, 1, acc, 16384, 16384, ctypes.byref(got))
        assert (got.rows, got.split) == (8, 2)
    lib.bwla_get_config(L.OP_DOT, 1, 0, 0, 1 << 24, ctypes.byref(got))
    assert (got.block, got.unroll, got.grid, got.increment) == (1024, 4, 256, 0)
    lib.bwla_get_config(L.OP_DOT, 1, 1, 0, 1 << 24, ctypes.byref(got))
    assert (got.block, got.unroll, got.grid, got.increment) == (256, 2, 512, 1)
    # malformed: a bad block, a bad mode, the old ten-column layout; nothing is installed
    for text in ("1 0 -1 -1 500 2 2 0 0 0 0\n", "1 0 2 -1 512 2 2 0 0 0 0\n", "1 0 -1 512 2 2 0 0 0 0\n",
                 "1 0 -1 -1 128 2 2 0 0 0 0\n1 0 -1 -1 500 2 2 0 0 0 0\n"):
        p.write_text(text)
        assert lib.bwla_load_tuning(str(p).encode()) == L.ERR_INVALID_ARG, text
        lib.bwla_get_config(L.OP_AXPBY, 0, 0, 0, 1 << 20, ctypes.byref(got))
        assert got.block == 512
    assert lib.bwla_load_tuning(b"/nonexistent/file") == L.ERR_INVALID_ARG
    for op in range(L.OP_COUNT):
        for t in range(3):
            lib.bwla_set_config(op, t, -1, -1, None)


def test_batch_plan_validation(L):
    lib = L.lib
    h = ctypes.c_void_p()
    g = (L.GemvDesc * 1)(L.GemvDesc(FAKE, 10, 20, 19, FAKE + (1 << 30), FAKE + (1 << 31)))
    d = (L.DotDesc * 1)()
    assert lib.bwla_batch_plan_create(0, 0, 0, g, 1, d, 0, None, ctypes.byref(h)) == L.ERR_INVALID_ARG
    assert not h.value
    d = (L.DotDesc * 1)(L.DotDesc(FAKE, FAKE, 10, None))
    assert lib.bwla_batch_plan_create(0, 0, 0, g, 0, d, 1, None, ctypes.byref(h)) == L.ERR_INVALID_ARG
    assert lib.bwla_batch_plan_create(0, 0, 1, g, 0, d, 0, None, ctypes.byref(h)) == L.ERR_UNSUPPORTED
    big = L.Config(block=1024)  # the batched work-groups hold at most 512 threads
    assert lib.bwla_batch_plan_create(0, 0, 0, g, 0, d, 0, ctypes.byref(big), ctypes.byref(h)) == L.ERR_INVALID_ARG
    assert "512" in lib.bwla_last_error().decode()
    assert lib.bwla_batch_run(None, None) == L.ERR_INVALID_ARG
    assert lib.bwla_batch_replay(None, None) == L.ERR_INVALID_ARG


def test_persistent_batch_is_refused(L, monkeypatch):
    """The persistent work-queue kernel is switched off: asking for it fails
    plan creation before any allocation or launch (the getenv is read at
    every creation)."""
    lib = L.lib
    h = ctypes.c_void_p()
    g = (L.GemvDesc * 1)()
    d = (L.DotDesc * 1)()
    monkeypatch.setenv("BWLA_ENABLE_UNVALIDATED_BATCH", "1")
    assert lib.bwla_batch_plan_create(0, 0, 0, g, 0, d, 0, None, ctypes.byref(h)) == L.ERR_UNSUPPORTED
    assert "switched off" in lib.bwla_last_error().decode()
    assert not h.value


def test_host_sizing_never_crashes_on_degenerate_shapes(L):
    """Workspace sizing and configuration resolution are host arithmetic; sweep
    them over empty, tiny and huge shapes for every op, layout and dtype."""
    lib = L.lib
    b = ctypes.c_size_t()
    c = L.Config()
    dims = [0, 1, 2, 3, 63, 64, 65, 4096, 1 << 20, (1 << 31) + 7]
    for t in range(3):
        for m in dims:
            for n in dims:
                for layout in (0, 1):
                    for trans in (0, 1):
                        for op in (L.OP_GEMV_ROWS, L.OP_GEMV_COLS):
                            assert lib.bwla_workspace_size(op, t, 0, layout, trans, m, n, ctypes.byref(b)) == L.OK
                assert lib.bwla_workspace_size(L.OP_DOT, t, 0, 0, 0, 0, n, ctypes.byref(b)) == L.OK
                for op in range(L.OP_COUNT):
                    for acc in (0, 1):
                        assert lib.bwla_get_config(op, t, acc, m, n, ctypes.byref(c)) == L.OK
                        assert c.block >= 64 and c.vec >= 1 and c.split >= 1


def test_empty_gemv_needs_no_workspace(L):
    b = ctypes.c_size_t(123)
    assert L.lib.bwla_workspace_size(L.OP_GEMV_ROWS, 0, 0, 0, 0, 0, 6, ctypes.byref(b)) == L.OK
    assert b.value == 0
    assert L.lib.bwla_workspace_size(L.OP_GEMV_ROWS, 0, 0, 0, 0, 4, 0, ctypes.byref(b)) == L.OK
    assert b.value == 0


def test_gemv_dot_validation(L):
    """bwla_gemv_dot: argument errors are caught before anything is enqueued."""
    lib = L.lib
    A, x, y, w, d = FAKE, FAKE + (1 << 30), FAKE + (2 << 30), FAKE + (3 << 30), FAKE + (4 << 30)
    ws = FAKE + (5 << 30)
    big = 1 << 24
    # bf16 storage has no bf16 GEMV output
    assert lib.bwla_gemv_dot(2, 0, 0, 0, 10, 20, A, 20, x, y, w, 1, d, ws, big, None) == L.ERR_UNSUPPORTED
    # dot type: f32 inner product of f64 data is not offered
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 10, 20, A, 20, x, y, w, 1, d, ws, big, None) == L.ERR_UNSUPPORTED
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 10, 20, A, 20, x, y, w, 0, None, ws, big, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 10, 20, A, 20, x, y, None, 0, d, ws, big, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 10, 20, A, 19, x, y, w, 0, d, ws, big, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot(0, 0, 0, 2, 10, 20, A, 20, x, y, w, 0, d, ws, big, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot(0, 5, 0, 0, 10, 20, A, 20, x, y, w, 0, d, ws, big, None) == L.ERR_UNSUPPORTED
    # overlaps: y with w, dot with y, dot with w, dot inside A, y inside x
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 10, 20, A, 20, x, y, y + 8, 0, d, ws, big, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 10, 20, A, 20, x, y, w, 0, y + 16, ws, big, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 10, 20, A, 20, x, y, w, 0, w, ws, big, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 10, 20, A, 20, x, y, w, 0, A + 80, ws, big, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 10, 20, A, 20, x, x + 8, w, 0, d, ws, big, None) == L.ERR_INVALID_ARG
    # w may alias x (both read only): only the workspace is missing here
    assert lib.bwla_gemv_dot(0, 0, 0, 0, 20, 20, A, 20, x, y, x, 0, d, None, 0, None) == L.ERR_WORKSPACE


def test_gemv_dot_workspace_size(L):
    lib = L.lib
    b, g = ctypes.c_size_t(), ctypes.c_size_t()
    for t in (0, 1):
        for layout in (0, 1):
            for trans in (0, 1):
                for (m, n) in [(1, 1), (37, 3000), (3000, 37), (8192, 8192), (16384, 16384)]:
                    assert lib.bwla_gemv_dot_workspace_size(t, layout, trans, m, n, ctypes.byref(b)) == L.OK
                    assert lib.bwla_workspace_size(L.OP_GEMV_ROWS, t, 0, layout, trans, m, n,
                                                   ctypes.byref(g)) == L.OK
                    # the epilogue adds at least one float64 pair to the GEMV's own partials
                    assert b.value >= g.value + 16, (t, layout, trans, m, n)
                    assert b.value % 16 == 0
    assert lib.bwla_gemv_dot_workspace_size(0, 0, 0, 0, 5, ctypes.byref(b)) == L.OK and b.value == 0
    assert lib.bwla_gemv_dot_workspace_size(0, 0, 0, 5, 0, ctypes.byref(b)) == L.OK and b.value == 0
    assert lib.bwla_gemv_dot_workspace_size(0, 0, 0, -1, 5, ctypes.byref(b)) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot_workspace_size(0, 3, 0, 1, 5, ctypes.byref(b)) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_dot_workspace_size(0, 0, 0, 1, 5, None) == L.ERR_INVALID_ARG


def test_dot_noalloc_validation(L):
    """The no-workspace inner product validates like bwla_dot before any HIP
    call (these run without a GPU)."""
    lib = L.lib
    X, Y, O = FAKE, FAKE + (1 << 30), FAKE + (2 << 30)
    assert lib.bwla_dot_noalloc(0, 0, -1, X, Y, 0, O, None) == L.ERR_INVALID_ARG
    assert lib.bwla_dot_noalloc(9, 0, 10, X, Y, 0, O, None) == L.ERR_UNSUPPORTED
    assert lib.bwla_dot_noalloc(0, 4, 10, X, Y, 0, O, None) == L.ERR_UNSUPPORTED      # accumulation mode
    assert lib.bwla_dot_noalloc(0, 0, 10, X, Y, 1, O, None) == L.ERR_UNSUPPORTED      # f32 out of f64 data
    assert lib.bwla_dot_noalloc(1, 0, 10, X, Y, 2, O, None) == L.ERR_UNSUPPORTED      # bf16 output
    assert lib.bwla_dot_noalloc(0, 0, 10, X, Y, 0, None, None) == L.ERR_INVALID_ARG
    assert lib.bwla_dot_noalloc(0, 0, 10, None, Y, 0, O, None) == L.ERR_INVALID_ARG
    assert lib.bwla_dot_noalloc(0, 0, 10, X, Y, 0, X + 16, None) == L.ERR_INVALID_ARG  # out inside x


def test_strided_validation(L):
    """Increments: zero output increments, overlaps and oversize strides are
    caught before anything is enqueued.  Every call here fails validation
    (none may reach a launch with these placeholder addresses)."""
    lib = L.lib
    X, Y, Z = FAKE, FAKE + (1 << 30), FAKE + (2 << 30)
    assert lib.bwla_copy_strided(0, 10, Y, 1, X, 0, None) == L.ERR_INVALID_ARG        # output inc 0
    assert lib.bwla_copy_strided(0, -1, Y, 1, X, 1, None) == L.ERR_INVALID_ARG
    assert lib.bwla_copy_strided(5, 10, Y, 1, X, 2, None) == L.ERR_UNSUPPORTED
    assert lib.bwla_copy_strided(0, 0, None, 3, None, 2, None) == L.OK               # empty
    assert lib.bwla_copy_strided(0, 10, None, 2, X, 2, None) == L.ERR_INVALID_ARG
    # same elements, opposite directions: not an exact alias
    assert lib.bwla_copy_strided(0, 10, X, -2, X, 2, None) == L.ERR_INVALID_ARG
    # interleaved f64 vectors 8 bytes apart with stride 2 share no element,
    # but stride 2 vectors 4 bytes apart do
    assert lib.bwla_copy_strided(0, 10, X + 4, 2, X, 2, None) == L.ERR_INVALID_ARG
    assert lib.bwla_copy_strided(0, 1 << 40, X, 1 << 30, Y, 1, None) == L.ERR_INVALID_ARG  # too large
    assert lib.bwla_axpby_strided(0, 10, 1.0, None, Y, 2, 1.0, None, Z, 3, X, 0, None) == L.ERR_INVALID_ARG
    assert lib.bwla_axpby_strided(0, 10, 1.0, None, X + 4, 3, 1.0, None, Z, 3, X, 3, None) == L.ERR_INVALID_ARG
    assert lib.bwla_axpby_strided(0, 10, 1.0, X + 16, Y, 2, 1.0, None, Z, 2, X, 2, None) == L.ERR_INVALID_ARG
    assert lib.bwla_scal(0, 10, 2.0, None, X, 0, None) == L.ERR_INVALID_ARG
    assert lib.bwla_scal(0, 10, 2.0, None, None, 1, None) == L.ERR_INVALID_ARG
    assert lib.bwla_scal(0, 10, 2.0, X + 8, X, 1, None) == L.ERR_INVALID_ARG          # device scalar inside x
    assert lib.bwla_scal(0, 0, 2.0, None, None, 0, None) == L.OK
    # out-of-place scaling (unit increments): exact aliasing only
    assert lib.bwla_scal_to(0, -1, 2.0, None, Y, X, None) == L.ERR_INVALID_ARG
    assert lib.bwla_scal_to(6, 10, 2.0, None, Y, X, None) == L.ERR_UNSUPPORTED
    assert lib.bwla_scal_to(0, 10, 2.0, None, None, X, None) == L.ERR_INVALID_ARG
    assert lib.bwla_scal_to(0, 10, 2.0, None, Y, None, None) == L.ERR_INVALID_ARG
    assert lib.bwla_scal_to(0, 10, 2.0, None, X + 8, X, None) == L.ERR_INVALID_ARG    # partial overlap
    assert lib.bwla_scal_to(1, 10, 2.0, X + 36, Y, X, None) == L.ERR_INVALID_ARG      # device scalar inside x
    assert lib.bwla_scal_to(0, 0, 2.0, None, None, None, None) == L.OK
    ws = FAKE + (3 << 30)
    for fn, args in ((lib.bwla_dot_strided, (X, 2, Y, -3)), ):
        assert fn(0, 0, 10, *args, 0, X + 8, ws, 1 << 20, None) == L.ERR_INVALID_ARG  # out inside x's span
        assert fn(0, 0, 10, *args, 1, Z, ws, 1 << 20, None) == L.ERR_UNSUPPORTED      # f32 out of f64 data
        assert fn(0, 0, 10, *args, 0, None, ws, 1 << 20, None) == L.ERR_INVALID_ARG
    assert lib.bwla_nrm2_strided(0, 0, 10, X, -2, 0, X + 16, ws, 1 << 20, None) == L.ERR_INVALID_ARG
    assert lib.bwla_asum(0, 3, 10, X, 1, 0, Z, ws, 1 << 20, None) == L.ERR_UNSUPPORTED  # accumulation mode
    assert lib.bwla_asum(0, 0, 10, X, 1, 0, X + 40, ws, 1 << 20, None) == L.ERR_INVALID_ARG
    # a large strided reduction needs its partials
    assert lib.bwla_asum(0, 0, 1 << 24, X, 2, 0, Z, None, 0, None) == L.ERR_WORKSPACE


def test_gemv_ex_validation_and_workspace(L):
    lib = L.lib
    A, x, y, ws = FAKE, FAKE + (1 << 30), FAKE + (2 << 30), FAKE + (3 << 30)
    args = (0, 0, 0, 0, 10, 20, 2.0, A, 20)
    assert lib.bwla_gemv_ex(*args, x, 2, 1.0, 0, y, 0, ws, 1 << 20, None) == L.ERR_INVALID_ARG    # incy 0
    assert lib.bwla_gemv_ex(*args, x, 2, 1.0, 1, y, 1, ws, 1 << 20, None) == L.ERR_UNSUPPORTED    # f32 out, f64
    assert lib.bwla_gemv_ex(*args, x, 2, 1.0, 0, None, 1, ws, 1 << 20, None) == L.ERR_INVALID_ARG
    assert lib.bwla_gemv_ex(*args, x, 2, 1.0, 0, x + 8, 1, ws, 1 << 20, None) == L.ERR_INVALID_ARG  # y in x
    assert lib.bwla_gemv_ex(*args, x, 2, 1.0, 0, A + 16, 3, ws, 1 << 20, None) == L.ERR_INVALID_ARG  # y in A
    assert lib.bwla_gemv_ex(*args, x, 2, 1.0, 0, y, 1, None, 0, None) == L.ERR_WORKSPACE
    assert lib.bwla_gemv_ex(0, 0, 0, 0, 0, 20, 2.0, A, 20, x, 2, 1.0, 0, None, 1, None, 0, None) == L.OK
    b, g = ctypes.c_size_t(), ctypes.c_size_t()
    for t, ot in ((0, 0), (1, 1), (1, 0), (2, 1)):
        for layout in (0, 1):
            for trans in (0, 1):
                for (m, n) in [(1, 1), (37, 3000), (16384, 16384)]:
                    assert lib.bwla_gemv_ex_workspace_size(t, ot, layout, trans, m, n, ctypes.byref(b)) == L.OK
                    assert lib.bwla_workspace_size(L.OP_GEMV_ROWS, t, 0, layout, trans, m, n,
                                                   ctypes.byref(g)) == L.OK
                    out_len, in_len = (n, m) if trans else (m, n)
                    es, os_ = (8, 4, 2)[t], (8 if ot == 0 else 4)
                    assert b.value >= g.value + out_len * os_ + in_len * es
    assert lib.bwla_gemv_ex_workspace_size(2, 2, 0, 0, 5, 5, ctypes.byref(b)) == L.ERR_UNSUPPORTED
    assert lib.bwla_gemv_ex_workspace_size(0, 0, 0, 0, 0, 5, ctypes.byref(b)) == L.OK and b.value == 0


def test_gemv_split_keeps_a_tuned_work_group_count(L):
    """With split 0 and a nonzero grid, a GEMV entry keeps its work-group
    count on every aspect ratio: split = ceil(grid / output tiles).  An
    explicit split stays fixed."""
    lib = L.lib
    got = L.Config()
    try:
        assert lib.bwla_set_config(L.OP_GEMV_COLS, 1, -1, -1,
                                   ctypes.byref(L.Config(block=512, vec=2, unroll=8, grid=256))) == L.OK
        # (lines, line length): tiles of 64 * vec = 128 outputs
        for lines, length, split in ((4096, 4096, 8), (16384, 2048, 16), (2048, 16384, 2), (40, 4096, 5)):
            assert lib.bwla_get_config(L.OP_GEMV_COLS, 1, 0, lines, length, ctypes.byref(got)) == L.OK
            assert got.split == split, (lines, length, got.split)
            assert got.grid == -(-length // 128) * split
        assert lib.bwla_set_config(L.OP_GEMV_ROWS, 1, -1, -1,
                                   ctypes.byref(L.Config(block=512, vec=4, rows=8, grid=512))) == L.OK
        for lines, length, split in ((4096, 4096, 1), (2048, 16384, 2), (16384, 2048, 1), (512, 16384, 8)):
            assert lib.bwla_get_config(L.OP_GEMV_ROWS, 1, 0, lines, length, ctypes.byref(got)) == L.OK
            assert got.split == split, (lines, length, got.split)
            assert got.grid == -(-lines // 8) * split
        assert lib.bwla_set_config(L.OP_GEMV_ROWS, 1, -1, -1,
                                   ctypes.byref(L.Config(block=512, vec=4, rows=8, split=3, grid=512))) == L.OK
        lib.bwla_get_config(L.OP_GEMV_ROWS, 1, 0, 2048, 16384, ctypes.byref(got))
        assert got.split == 3
    finally:
        for op in (L.OP_GEMV_ROWS, L.OP_GEMV_COLS):
            lib.bwla_set_config(op, 1, -1, -1, None)


def test_rows_block_fits_the_line(L):
    """A rows-GEMV work-group never holds more threads than one slice of a
    line has packs (rounded up to 64), whatever the table says."""
    lib = L.lib
    got = L.Config()
    assert lib.bwla_set_config(L.OP_GEMV_ROWS, 1, -1, -1,
                               ctypes.byref(L.Config(block=1024, vec=4, rows=2, split=1))) == L.OK
    try:
        for n, want in ((2048, 512), (16384, 1024), (100, 64), (4096, 1024), (4100, 1024)):
            assert lib.bwla_get_config(L.OP_GEMV_ROWS, 1, 0, 16384, n, ctypes.byref(got)) == L.OK
            assert got.block == want, (n, got.block)
    finally:
        lib.bwla_set_config(L.OP_GEMV_ROWS, 1, -1, -1, None)

