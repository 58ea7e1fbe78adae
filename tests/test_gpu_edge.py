"""GPU edge cases of the boundary.

* The plain three-call path launched over uneven sub-ranges of subdomains
  (one caller owning several subdomains per call, and one call per
  subdomain), including empty ranges, is bitwise the fused step: the
  sub-range arguments only select which segments a call works on.
* Pools without particles (every segment empty) step to empty pools with
  no flags, through the fused, plain and per-stage paths.
"""
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


def c2s_case():
    c = Case("C2S", 60000, 32, (4, 4, 4))
    c.params = pm.Params(min(c.dt, 0.015), c.g)
    return c


def fused_reference(c):
    pin = c.pin()
    send, out = c.send(), c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.step(c.field, c.dc, pin, out, send, c.params)
    assert ctx.get_status() == 0
    return ctx, pin.size, out, send


# (advance ranges, classify ranges, compact ranges) as [first, end) pairs over 64
RANGES = {
    "uneven": ([(0, 5), (5, 6), (6, 6), (6, 40), (40, 64)],
               [(0, 1), (1, 33), (33, 63), (63, 64)],
               [(0, 17), (17, 18), (18, 18), (18, 64)]),
    "one per subdomain": ([(s, s + 1) for s in range(64)],
                          [(s, s + 1) for s in range(64)],
                          [(s, s + 1) for s in range(64)]),
}


@pytest.mark.parametrize("split", list(RANGES))
def test_subdomain_ranges_equal_the_fused_step(split):
    say(f"[test] plain path over sub-ranges: {split}")
    c = c2s_case()
    assert c.dc.nsub == 64
    ctx, size, out_a, send_a = fused_reference(c)
    adv, cls, cmp = RANGES[split]
    work = c.pin()
    send_b, out_b = c.send(), c.pout(size)
    for s0, s1 in adv:
        ctx.interp_advance(c.field, work, c.params, s0, s1 - s0)
    for s0, s1 in cls:
        ctx.classify_scan_pack(c.dc, work, send_b, s0, s1 - s0)
    for s0, s1 in cmp:
        ctx.compact_append(c.dc, work, send_b, out_b, s0, s1 - s0)
    assert ctx.get_status() == 0
    say(f"  migrants {int(send_b.to_host().count.sum())}")
    assert_same_device_pools(out_a, out_b, c.dc.nsub, f"out ({split})")
    assert_same_device_pools(send_a, send_b, c.dc.nsub * 27, f"send ({split})")


@pytest.mark.parametrize("path", ["fused", "plain", "staged"])
def test_pool_without_particles(path):
    say(f"[test] empty pool, {path} path")
    c = c2s_case()
    host = c.host
    vdt = np.float32 if c.mode == "mixed" else np.float64
    empty = gen.empty_pool(host.base, host.cap, vdt)
    dev = c.dev
    pin = pm.DevicePool.from_host(empty, dev)
    send, out = c.send(), c.pout(pin.size)
    # non-zero counts in the outputs must be overwritten
    out.count.fill_(7)
    send.count.fill_(7)
    ctx = c.ctx(pin, send)
    if path == "fused":
        ctx.step(c.field, c.dc, pin, out, send, c.params)
    elif path == "plain":
        ctx.interp_advance(c.field, pin, c.params)
        ctx.classify_scan_pack(c.dc, pin, send)
        ctx.compact_append(c.dc, pin, send, out)
    else:
        mid = pm.DeviceStagePool.empty(host.base, host.cap, vdtype=c.vdt, device=dev,
                                       size=pin.size)
        msend = pm.DeviceStagePool.empty(c.sb, c.sc, vdtype=c.vdt, device=dev,
                                         size=send.size)
        ctx.step_staged(c.field, c.dc, pin, mid, msend, out, send, c.params)
        assert int(mid.count.sum().item()) == 0
        assert int(msend.count.sum().item()) == 0
    assert ctx.get_status() == 0
    assert int(out.count.sum().item()) == 0
    assert int(send.count.sum().item()) == 0


@pytest.mark.parametrize("path,mode,drag", [("fused", "f64", "stokes"),
                                            ("fused", "mixed", "nonlinear"),
                                            ("staged", "f64", "nonlinear")])
def test_zero_time_step_is_the_identity(path, mode, drag):
    """dt = 0: X' = X + 0 and V' = V + 0 exactly, nobody leaves, and the
    stable compaction keeps every segment's order, so out is in bitwise."""
    say(f"[test] dt = 0, {path} {mode} {drag}")
    c = Case("C2S", 30000, 32, (4, 4, 4), mode=mode, drag=drag)
    c.params = pm.Params(0.0, c.g, drag=drag)
    pin = c.pin()
    send, out = c.send(), c.pout(pin.size)
    ctx = c.ctx(pin, send)
    if path == "fused":
        ctx.step(c.field, c.dc, pin, out, send, c.params)
    else:
        mid = pm.DeviceStagePool.empty(c.host.base, c.host.cap, vdtype=c.vdt, device=c.dev,
                                       size=pin.size)
        msend = pm.DeviceStagePool.empty(c.sb, c.sc, vdtype=c.vdt, device=c.dev,
                                         size=send.size)
        ctx.step_staged(c.field, c.dc, pin, mid, msend, out, send, c.params)
        assert int(msend.count.sum().item()) == 0
    assert ctx.get_status() == 0
    assert int(send.count.sum().item()) == 0
    assert_same_device_pools(out, pin, c.dc.nsub, f"dt=0 {path} {mode}")
