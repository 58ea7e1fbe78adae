"""GPU parity of the nonlinear drag law (Sect. 2.2: f = 1 + 0.15 Re_p^0.687,
Re_p = 2 r |V - U| / nu, r from tau = (2/9)(rho_p/rho) r^2 / nu; nu = 1.5e-5,
rho_p/rho = 843 in the units of the synthetic fields) against the oracle:
the in-place advance within 1e-12, the fused step with bit-exact migration,
and fused == plain bitwise.  Each case also checks that the law changes the
result, so a silently ignored drag flag fails."""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import Case, assert_same_device_pools, compare_pools, say, seg

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name,npart,n,p", [("C1", 20000, 32, (2, 2, 2)),
                                            ("C2", 30000, 32, (1, 1, 1))])
def test_nonlinear_advance_matches_oracle(name, npart, n, p):
    say(f"[test] nonlinear interp_advance {name}")
    c = Case(name, npart, n, p, drag="nonlinear")
    pin = c.pin()
    ctx = c.ctx(pin, c.send())
    ctx.interp_advance(c.field, pin, c.params)
    assert ctx.get_status() == 0
    got = pin.to_host()
    changed = 0.0
    for q in range(c.dc.nsub):
        s = seg(c.host, q)
        args = (c.ofield, c.host.x[:, s], c.host.v[:, s], c.host.tau[s], c.dt, c.g)
        xr, vr, _ = oracle.advance(*args, drag="nonlinear")
        _, vs, _ = oracle.advance(*args)
        ex = np.abs(got.x[:, s] - xr) / np.maximum(np.abs(xr), c.wl.L / c.wl.n)
        ev = np.abs(got.v[:, s] - vr) / max(1.0, np.abs(vr).max())
        assert ex.max() <= 1e-12 and ev.max() <= 1e-12, (ex.max(), ev.max())
        changed = max(changed, float(np.abs(vr - vs).max()))
    say(f"  max |V_nonlinear - V_stokes| {changed:.2e}")
    assert changed > 1e-6


@pytest.mark.parametrize("name,npart,n,p", [("C1", None, None, None),
                                            ("C2", 40000, 32, None),
                                            ("C3", 50000, 32, (4, 4, 4))])
def test_nonlinear_step_matches_oracle(name, npart, n, p):
    say(f"[test] nonlinear step {name}")
    c = Case(name, npart, n, p, drag="nonlinear")
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.step(c.field, c.dc, pin, pout, send, c.params)
    flags = ctx.get_status()
    ref_out, ref_send, _, oflags = c.oracle_step()
    assert flags == oflags == 0
    delta = c.wl.L / c.wl.n
    compare_pools(send.to_host(), ref_send, c.dc.nsub * 27, c.wl.L, delta, what="send")
    ex, ev = compare_pools(pout.to_host(), ref_out, c.dc.nsub, c.wl.L, delta, what="out")
    say(f"  migrants {int(ref_send.count.sum())}; max err x {ex:.2e} v {ev:.2e}")


def test_nonlinear_fused_equals_plain_bitwise():
    say("[test] nonlinear fused == plain")
    c = Case("C2S", 80000, 32, (8, 8, 8), drag="nonlinear")
    c.params.dt = min(c.dt, 0.015)
    pin = c.pin()
    send_a, send_b = c.send(), c.send()
    out_a, out_b = c.pout(pin.size), c.pout(pin.size)
    ctx = c.ctx(pin, send_a)
    ctx.step(c.field, c.dc, pin, out_a, send_a, c.params)
    plain_in = c.pin()
    ctx.interp_advance(c.field, plain_in, c.params)
    ctx.classify_scan_pack(c.dc, plain_in, send_b)
    ctx.compact_append(c.dc, plain_in, send_b, out_b)
    assert ctx.get_status() == 0
    assert_same_device_pools(out_a, out_b, c.dc.nsub, "out")
    assert_same_device_pools(send_a, send_b, c.dc.nsub * 27, "send")


def test_bad_drag_parameters_are_argument_errors():
    from paper_2604_11008_amd import pm
    c = Case("C1", 2000, 16, (1, 1, 1))
    pin = c.pin()
    ctx = c.ctx(pin, c.send())
    for kw in (dict(drag="nonlinear", nu=0.0), dict(drag="nonlinear", density_ratio=-1.0),
               dict(drag="nonlinear", nu=float("nan"))):
        with pytest.raises(pm.PMError, match="nonlinear drag"):
            ctx.interp_advance(c.field, pin, pm.Params(c.dt, c.g, **kw))


def test_default_launch_shape_follows_the_variant():
    """256 x 4 by default for either drag law (256 x 2 only for the mixed
    kernels on an interleaved periodic field); a set shape until it is reset;
    fewer records per thread when the context's pool extent gives fewer than
    two tiles per compute unit."""
    from paper_2604_11008_amd import pm
    say("[test] per-variant default shapes")
    c = Case("C3", 50000, 32, (4, 4, 4), drag="nonlinear")
    send = c.send()
    stokes = pm.Params(c.dt, c.g)
    # the same particles in pools padded to a large extent
    extent = 1 << 22
    pin = pm.DevicePool.from_host(c.host, c.dev, size=extent)
    pout = c.pout(extent)
    big = pm.Context(extent, send.size, c.dc.nsub, device=c.dev)
    big.step(c.field, c.dc, pin, pout, send, c.params)
    assert big.get_tuning()[:2] == (256, 4)
    big.step(c.field, c.dc, pin, pout, send, stokes)
    assert big.get_tuning()[:2] == (256, 4)
    big.set_tuning(256, 1)
    big.step(c.field, c.dc, pin, pout, send, c.params)
    assert big.get_tuning()[:2] == (256, 1)
    big.set_tuning(0, 0)
    big.step(c.field, c.dc, pin, pout, send, c.params)
    assert big.get_tuning()[:2] == (256, 4)
    assert big.get_status() == 0
    # the unpadded pool (about 1.2e5 records) gives fewer than two
    # 256-record tiles per CU
    spin = c.pin()
    spout = c.pout(spin.size)
    small = c.ctx(spin, send)
    small.step(c.field, c.dc, spin, spout, send, stokes)
    assert small.get_tuning()[:2] == (256, 1)
    assert small.get_status() == 0


@pytest.mark.parametrize("drag,stagger", [("nonlinear", False), ("stokes", True)])
def test_periodic_variants_in_their_default_shape(drag, stagger):
    """The FP64 periodic nonlinear-drag and MAC kernels at 256 x 4 (their
    default for a large pool) against the oracle, and bitwise equal to 256 x 2,
    on a pool of many tiles per segment."""
    say(f"[test] periodic default shape drag={drag} stagger={stagger}")
    c = Case("C3", 600000, 64, (4, 4, 4), drag=drag, stagger=stagger)
    pin = c.pin()
    ctx = c.ctx(pin, c.send())
    outs = []
    for shape in ((256, 4), (256, 2)):
        ctx.set_tuning(*shape)
        send, pout = c.send(), c.pout(pin.size)
        ctx.step(c.field, c.dc, pin, pout, send, c.params)
        assert ctx.get_status() == 0
        assert tuple(ctx.get_tuning()[:2]) == shape
        outs.append((pout, send))
    assert_same_device_pools(outs[0][0], outs[1][0], c.dc.nsub, "out 256x4 vs 256x2")
    assert_same_device_pools(outs[0][1], outs[1][1], c.dc.nsub * 27, "send 256x4 vs 256x2")
    ref_out, ref_send, _, oflags = c.oracle_step()
    assert oflags == 0
    delta = c.wl.L / c.wl.n
    compare_pools(outs[0][1].to_host(), ref_send, c.dc.nsub * 27, c.wl.L, delta, what="send")
    ex, ev = compare_pools(outs[0][0].to_host(), ref_out, c.dc.nsub, c.wl.L, delta, what="out")
    say(f"  migrants {int(ref_send.count.sum())}; max err x {ex:.2e} v {ev:.2e}")
