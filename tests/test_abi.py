"""The C-ABI library loads (no GPU needed) and exports every function that
include/pm.h declares; the binding's structures match the header's layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("pm_interp_advance", "pm_classify_scan_pack", "pm_compact_append",
                     "pm_step", "pm_create", "pm_workspace_bytes", "pm_get_status"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2604_11008_amd import pm
    lib = ctypes.CDLL(pm.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_struct_layout_matches_header():
    from paper_2604_11008_amd import pm
    assert ctypes.sizeof(pm._Field) == 72
    assert ctypes.sizeof(pm._Decomp) == 40
    assert ctypes.sizeof(pm._Particles) == 96
    assert ctypes.sizeof(pm._Send) == 88
    assert ctypes.sizeof(pm._Params) == 32
    assert ctypes.sizeof(pm._Tuning) == 16


def test_host_only_calls():
    from paper_2604_11008_amd import pm
    lib = pm.lib()
    assert lib.pm_workspace_bytes(1 << 20, 1 << 16, 8) > (1 << 20) * 4 + (1 << 16) * 65
    assert lib.pm_workspace_bytes(-1, 0, 8) == 0
    h = ctypes.c_void_p()
    # argument errors are reported without touching a device
    assert lib.pm_create(ctypes.byref(h), None, 0, 100, 100, 0) == 1
    assert b"nsub" in lib.pm_last_error()
    assert lib.pm_create(None, None, 0, 100, 100, 1) == 1
