"""The C-ABI library loads (no GPU needed) and exports every function that
include/pm.h declares; the binding's structures match the header's layout."""
import ctypes
import os
import re
import subprocess

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


def header_layout(tmp_path):
    """sizeof and field offsets of the header's structs, from a C compiler."""
    probes = {
        "pm_field": ["n", "halo", "L", "dtype", "stagger", "u", "layout"],
        "pm_decomp": ["p", "bounds"],
        "pm_particles": ["nsub", "vdtype", "base", "cap", "count", "x", "v", "tau", "id"],
        "pm_sendbufs": ["base", "cap", "count", "x", "v", "tau", "id"],
        "pm_params": ["dt", "g", "drag", "nu", "density_ratio"],
        "pm_tuning": ["wg", "items", "blocks_per_cu", "xcd_block"],
        "pm_stage_particles": ["nsub", "vdtype", "base", "cap", "count", "x", "v", "xs", "vs",
                               "a", "tau", "id"],
        "pm_stage_sendbufs": ["base", "cap", "count", "x", "v", "xs", "vs", "a", "tau", "id"],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pm.h"', 'int main(void) {']
    for st, fields in probes.items():
        lines.append(f'printf("{st} sizeof %zu\\n", sizeof({st}));')
        for f in fields:
            lines.append(f'printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        st, f, v = line.split()
        res[(st, f)] = int(v)
    return probes, res


def test_binding_struct_layout_matches_header(tmp_path):
    from paper_2604_11008_amd import pm
    probes, ref = header_layout(tmp_path)
    cls = {"pm_field": pm._Field, "pm_decomp": pm._Decomp, "pm_particles": pm._Particles,
           "pm_sendbufs": pm._Send, "pm_params": pm._Params, "pm_tuning": pm._Tuning,
           "pm_stage_particles": pm._StageParticles, "pm_stage_sendbufs": pm._StageSend}
    for st, fields in probes.items():
        c = cls[st]
        assert ctypes.sizeof(c) == ref[(st, "sizeof")], st
        for f in fields:
            assert getattr(c, f).offset == ref[(st, f)], (st, f)


def test_host_only_calls():
    from paper_2604_11008_amd import pm
    lib = pm.lib()
    # a stayer slot per pool record and a 137-byte staging slot per send slot
    assert lib.pm_workspace_bytes(1 << 20, 1 << 16, 8) > (1 << 20) * 4 + (1 << 16) * 137
    assert lib.pm_workspace_bytes(-1, 0, 8) == 0
    assert lib.pm_workspace_bytes(1 << 35, 0, 8) == 0
    assert lib.pm_workspace_bytes(100, 1 << 35, 8) == 0
    assert lib.pm_workspace_bytes(100, 100, 4097) == 0
    # the re-sort: two (8-byte key, 4-byte position) buffers per pool record
    assert lib.pm_sort_workspace_bytes(1 << 20, 8) > (1 << 20) * 24
    assert lib.pm_sort_workspace_bytes(1 << 32, 8) == 0
    assert lib.pm_sort_workspace_bytes(-1, 8) == 0
    assert lib.pm_sort_workspace_bytes(100, 0) == 0
    assert lib.pm_sort(None, None, None, None, None, 0, None) == 1
    assert b"ctx" in lib.pm_last_error()
    h = ctypes.c_void_p()
    # argument errors are reported without touching a device
    assert lib.pm_create(ctypes.byref(h), None, 0, 100, 100, 0) == 1
    assert b"nsub" in lib.pm_last_error()
    assert lib.pm_create(None, None, 0, 100, 100, 1) == 1
    assert lib.pm_create(ctypes.byref(h), None, 0, 1 << 35, 100, 8) == 1
    assert b"extent" in lib.pm_last_error()


def test_binding_passes_the_row_pointers_of_each_array():
    """The structs handed to the library carry, for every (3, n) array, the
    addresses of its three rows (host tensors stand in for device ones)."""
    import numpy as np
    import torch
    from paper_2604_11008_amd import pm
    base = np.array([0, 40, 90], dtype=np.int64)
    cap = np.array([40, 50, 30], dtype=np.int64)
    for vdt in (torch.float64, torch.float32):
        p = pm.DevicePool.empty(base, cap, vdtype=vdt, device="cpu", size=130)
        pc, sc = p.particles(), p.sendbufs()
        for name in ("x", "v"):
            want = [getattr(p, name)[a].data_ptr() for a in range(3)]
            assert [getattr(pc, name)[a] for a in range(3)] == want
            assert [getattr(sc, name)[a] for a in range(3)] == want
        st = pm.DeviceStagePool.empty(base, cap, vdtype=vdt, device="cpu", size=130)
        spc, ssc = st.stage_particles(), st.stage_sendbufs()
        for name in ("x", "v", "xs", "vs", "a"):
            want = [getattr(st, name)[a].data_ptr() for a in range(3)]
            assert [getattr(spc, name)[a] for a in range(3)] == want
            assert [getattr(ssc, name)[a] for a in range(3)] == want


def test_noalloc_argument_errors_without_a_device():
    """pm_step_noalloc checks its flags pointer, subdomain count and the size
    of the scratch its extents need before it touches a device."""
    from paper_2604_11008_amd import pm
    lib = pm.lib()
    parts = pm._Particles()
    parts.nsub = 8
    one = ctypes.c_uint32()
    assert lib.pm_step_noalloc(None, None, ctypes.byref(parts), None, None, None, 100, 100,
                               None, None) == 1
    assert b"flags" in lib.pm_last_error()
    # 10^6 send-buffer records need about 137 MB of scratch, more than its 64 MiB
    assert lib.pm_step_noalloc(None, None, ctypes.byref(parts), None, None, None, 1 << 20,
                               1_000_000, ctypes.byref(one), None) == 1
    assert b"scratch" in lib.pm_last_error()
    parts.nsub = 0
    assert lib.pm_step_noalloc(None, None, ctypes.byref(parts), None, None, None, 100, 100,
                               ctypes.byref(one), None) == 1
    assert b"nsub" in lib.pm_last_error()


def test_binding_marshals_an_interleaved_field():
    """An interleaved field reaches the library as u[0] = its one array,
    u[1] = u[2] = NULL and layout 1; sizes that do not hold three values per
    stored node, and an interleaved MAC field, are refused (host tensors
    stand in for device ones)."""
    import pytest
    import torch
    from paper_2604_11008_amd import pm
    n, halo = (6, 5, 4), 1
    nodes = 8 * 7 * 6
    w = torch.zeros((nodes, 3), dtype=torch.float64)
    f = pm.DeviceField(w, n, halo, 1.0, device="cpu", interleaved=True)
    assert f.c.layout == pm.LAYOUT_INTERLEAVED == 1
    assert f.c.u[0] == w.data_ptr() and f.c.u[1] is None and f.c.u[2] is None
    split = pm.DeviceField([torch.zeros(nodes)] * 3, n, halo, 1.0, device="cpu")
    assert split.c.layout == pm.LAYOUT_SPLIT == 0
    with pytest.raises(pm.PMError):
        pm.DeviceField(torch.zeros(3 * nodes - 1, dtype=torch.float64), n, halo, 1.0,
                       device="cpu", interleaved=True)
    with pytest.raises(pm.PMError):
        pm.DeviceField(w, n, halo, 1.0, device="cpu", interleaved=True, stagger=True)


def test_interleave_argument_errors_without_a_device():
    """pm_field_interleave checks its field and output before any launch: a
    NULL field, a field already interleaved, a MAC field, a NULL output, an
    output overlapping a component, an unknown output type and a widening
    (host tensors stand in for device ones; no check reaches the device)."""
    import torch
    from paper_2604_11008_amd import pm
    lib = pm.lib()
    n, halo = (6, 5, 4), 1
    nodes = 8 * 7 * 6
    comps = [torch.zeros(nodes, dtype=torch.float64) for _ in range(3)]
    split = pm.DeviceField(comps, n, halo, 1.0, device="cpu")
    out = torch.zeros(3 * nodes, dtype=torch.float64)
    assert lib.pm_field_interleave(None, 0, out.data_ptr(), None) == 1
    assert b"field is NULL" in lib.pm_last_error()
    ilv = pm.DeviceField(out, n, halo, 1.0, device="cpu", interleaved=True)
    assert lib.pm_field_interleave(ctypes.byref(ilv.c), 0, out.data_ptr(), None) == 1
    assert b"one array per component" in lib.pm_last_error()
    mac = pm.DeviceField(comps, n, halo, 1.0, device="cpu", stagger=True)
    assert lib.pm_field_interleave(ctypes.byref(mac.c), 0, out.data_ptr(), None) == 1
    assert b"one array per component" in lib.pm_last_error()
    assert lib.pm_field_interleave(ctypes.byref(split.c), 0, None, None) == 1
    assert b"out is NULL" in lib.pm_last_error()
    big = torch.zeros(4 * nodes, dtype=torch.float64)
    shared = pm.DeviceField([big[:nodes], comps[1], comps[2]], n, halo, 1.0, device="cpu")
    assert lib.pm_field_interleave(ctypes.byref(shared.c), 0, big[nodes // 2:].data_ptr(),
                                   None) == 1
    assert b"overlaps field.u[0]" in lib.pm_last_error()
    assert lib.pm_field_interleave(ctypes.byref(split.c), 2, out.data_ptr(), None) == 1
    assert b"out_dtype" in lib.pm_last_error()
    split32 = pm.DeviceField([c.float() for c in comps], n, halo, 1.0, device="cpu")
    out32 = torch.zeros(3 * nodes, dtype=torch.float32)
    assert lib.pm_field_interleave(ctypes.byref(split32.c), 0, out32.data_ptr(), None) == 1
    assert b"does not widen" in lib.pm_last_error()
