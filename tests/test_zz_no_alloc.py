"""pm_step_noalloc (the fused step in the library's fixed device scratch, for
callers that cannot allocate) against pm_step (context and caller
workspace) through the C ABI: bitwise the same pools and send buffers, and
the same flags, on calls in a row with shrinking inputs, an overflowing
call, and the call after it."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_cases import Case, assert_same_device_pools, say
from paper_2604_11008_amd import gen, pm

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(name, npart, n, p, mode=None):
    c = Case(name, npart, n, p, mode=mode)
    if name == "C2S":
        c.params = pm.Params(0.015, c.g)
    # send buffers small enough for the fixed scratch (about 137 bytes per
    # send-buffer record)
    c.sb, c.sc = gen.send_layout(c.host.count, face=0.1, edge=0.03, corner=0.02, extra=32)
    return c


def _both(c, send_cap=None):
    """One step through pm_step and one through pm_step_noalloc from the
    same input; returns their outputs and flags."""
    sc = c.sc if send_cap is None else np.minimum(c.sc, send_cap)
    pin = c.pin()
    size = int((c.sb + c.sc).max())
    send_a = pm.DevicePool.empty(c.sb, sc, vdtype=c.vdt, device=c.dev, size=size)
    send_b = pm.DevicePool.empty(c.sb, sc, vdtype=c.vdt, device=c.dev, size=size)
    out_a, out_b = c.pout(pin.size), c.pout(pin.size)
    ctx = pm.Context(pin.size, send_a.size, c.dc.nsub, device=c.dev)
    ctx.step(c.field, c.dc, pin, out_a, send_a, c.params)
    fa = ctx.get_status()
    flags = torch.full((1,), -1, dtype=torch.int32, device=c.dev)
    pm.step_noalloc(c.field, c.dc, pin, out_b, send_b, c.params, flags)
    torch.cuda.synchronize()
    return (out_a, send_a, fa), (out_b, send_b, int(flags.item()))


@pytest.mark.parametrize("calls", [[("C2S", 60000, 32, (4, 4, 4), None),
                                    ("C1", 20000, 32, (2, 2, 2), None),
                                    ("C1", 5000, 16, (2, 2, 1), "mixed")]])
def test_noalloc_step_equals_pm_step(calls):
    for name, npart, n, p, mode in calls:
        say(f"[test] noalloc vs pm_step: {name} np={npart} n={n} p={p} mode={mode}")
        c = _case(name, npart, n, p, mode)
        (oa, sa, fa), (ob, sb, fb) = _both(c)
        assert fa == 0 and fb == 0, (fa, fb)
        assert_same_device_pools(ob, oa, c.dc.nsub, "out")
        assert_same_device_pools(sb, sa, c.dc.nsub * 27, "send")
        say(f"  equal: {int(oa.count.sum())} particles, {int(sa.count.sum())} migrants")


def test_noalloc_overflow_flags_then_a_clean_call():
    say("[test] noalloc overflow, then a clean call")
    c = _case("C2S", 40000, 32, (4, 4, 4))
    (oa, sa, fa), (ob, sb, fb) = _both(c, send_cap=1)
    assert fa & pm.SEND_OVERFLOW and fb == fa, (fa, fb)
    np.testing.assert_array_equal(sb.count.cpu().numpy(), sa.count.cpu().numpy())
    np.testing.assert_array_equal(ob.count.cpu().numpy(), oa.count.cpu().numpy())
    # the next call on the device starts without the previous call's flags
    (oa, sa, fa), (ob, sb, fb) = _both(c)
    assert fa == 0 and fb == 0, (fa, fb)
    assert_same_device_pools(ob, oa, c.dc.nsub, "out after overflow")


def test_noalloc_rejects_sizes_beyond_its_scratch():
    say("[test] noalloc size limit")
    c = _case("C1", 5000, 16, (2, 2, 2))
    pin, send = c.pin(), c.send()
    out = c.pout(pin.size)
    flags = torch.zeros(1, dtype=torch.int32, device=c.dev)
    lib = pm.lib()
    rc = lib.pm_step_noalloc(C.byref(c.field.c), C.byref(c.dc.c), C.byref(pin.particles()),
                             C.byref(out.particles()), C.byref(send.sendbufs()),
                             C.byref(c.params.c), pin.size, 1 << 24, flags.data_ptr(), None)
    assert rc == 1
    assert b"scratch" in lib.pm_last_error()
