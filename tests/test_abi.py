"""The C ABI library: it loads without a GPU, exports every entry point
include/rambo.h declares, and the Python binding names them all."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1910_04358_amd import rambo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rambo.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rambo_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(rambo.LIB_PATH):
        from paper_1910_04358_amd import build
        build.build()
    return rambo.lib()


def test_header_declares_the_boundary():
    names = declared()
    for f in ("rambo_create", "rambo_destroy", "rambo_insert", "rambo_insert_batch", "rambo_insert_seqs",
              "rambo_query_kmers", "rambo_query_seqs", "rambo_query_seqs_ids", "rambo_last_error", "rambo_sync"):
        assert f in names


def test_every_declared_symbol_is_exported(so):
    for name in declared():
        assert hasattr(so, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", rambo.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (rambo_\w+)", out))
    assert set(declared()) <= exported
    # nothing else of ours leaks out of the library
    assert exported <= set(declared()), exported - set(declared())


def test_binding_covers_the_header():
    assert set(declared()) <= set(rambo.SIGNATURES)


def test_invalid_create_reports_einval_without_touching_a_device(so):
    L = rambo.lib()
    assert not L.rambo_create(0, 10, 3, 1 << 20, 2, 1)
    assert L.rambo_last_status() == rambo.EINVAL
    assert b"out of range" in L.rambo_last_error()
    assert not L.rambo_create(100, 10, 9, 1 << 20, 2, 1)      # R > 8
    assert not L.rambo_create(100, 9000, 3, 1 << 20, 2, 1)    # B > 8192
    assert not L.rambo_create(100, 10, 3, 1 << 20, 0, 1)      # eta = 0
    assert not L.rambo_create(100, 10, 3, 1 << 20, 17, 1)     # eta > 16
    L.rambo_destroy(None)                                     # NULL-safe


def test_null_handle_calls_fail_cleanly(so):
    L = rambo.lib()
    assert L.rambo_insert(None, 0, None, 0) == rambo.EINVAL
    assert L.rambo_query_seqs(None, None, None, 0, None, None) == rambo.EINVAL
    assert L.rambo_set_mode(None, 0) == rambo.EINVAL
    assert L.rambo_result_words(None) == 0


def test_server_rejects_bad_config(so):
    L = rambo.lib()
    cfg = rambo.ServerConfig(0, 4, 100, 1000, 0, 10)  # zero budget
    assert not L.rambo_server_start(None, ctypes.byref(cfg))
    assert L.rambo_last_status() == rambo.EINVAL
    assert L.rambo_server_stop(None) == 0


def test_offsets_check():
    import numpy as np
    rambo.check_offsets(np.array([0, 3, 3, 10], dtype=np.uint64), 10)
    with pytest.raises(ValueError):
        rambo.check_offsets(np.array([0, 5, 3], dtype=np.uint64), 10)
    with pytest.raises(ValueError):
        rambo.check_offsets(np.array([0, 11], dtype=np.uint64), 10)
