"""The C-ABI library loads and exports every entry point include/emin.h
declares (no GPU needed: nothing is called that touches the device)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "emin.h")).read()
    return sorted(set(re.findall(r"\b(emin_[a-z0-9_]+)\s*\(", text)))


def test_header_lists_entry_points():
    syms = declared_symbols()
    for s in ("emin_pattern", "emin_setup", "emin_rap", "emin_pattern_destroy"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_1607_02489_amd import emin as E
    if not os.path.exists(E.LIBPATH):
        pytest.skip("libemin.so not built")
    lib = C.CDLL(E.LIBPATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert set(E.SYMBOLS) <= set(declared_symbols())
    E.lib()
    assert E.lib().emin_version().startswith(b"emin")
    assert E.lib().emin_status_string(6) == b"ERR_BREAKDOWN"


def test_null_arguments_rejected_without_device():
    from paper_1607_02489_amd import emin as E
    if not os.path.exists(E.LIBPATH):
        pytest.skip("libemin.so not built")
    L = E.lib()
    assert L.emin_pattern(None, None, None, None) == 1          # ERR_ARG
    s = E.c_sizes()
    assert L.emin_pattern_info(None, C.byref(s)) == 1
    assert L.emin_setup(None, None, None, None, None, None, None) == 1
    assert L.emin_rap(None, None, None, None, None, None, 0, None) == 1
    L.emin_pattern_destroy(None)                                   # NULL-safe
