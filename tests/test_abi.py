"""The C-ABI library loads and exports every symbol include/snn.h declares
(no GPU needed: nothing here runs a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include"))) if f.endswith(".h")]
LIB = os.path.join(ROOT, "paper_2301_10622_amd", "libsnn.so")


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"\b(snn_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("snn_create", "snn_destroy", "snn_insert", "snn_delete", "snn_search"):
        assert core in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libsnn.so not built"
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    import paper_2301_10622_amd as P

    assert set(declared_functions()) <= set(P.EXPORTS) | set(getattr(P, "EXTRA_EXPORTS", []))


def test_create_rejects_bad_config_without_touching_the_device():
    import paper_2301_10622_amd as P

    L = P.lib()
    out = ctypes.c_void_p()
    for cfg in (P.Config(0, 32, 1, 100, 0, 0, 0), P.Config(100, 0, 1, 100, 0, 0, 0), P.Config(100, 32, 5, 100, 0, 0, 0),
                P.Config(100, 32, 1, 0, 0, 0, 0), P.Config(100, 32, 1, 100, 0, 8, 0),
                P.Config(100, 1025, 1, 100, 0, 0, 0)):
        assert L.snn_create(ctypes.byref(cfg), None, ctypes.byref(out)) == -1
        assert not out.value
    assert L.snn_last_error(None) == b"null index"
    assert L.snn_live_count(None) == 0
