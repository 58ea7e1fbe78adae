"""GPU parity at full size, in the launch configuration the benchmark times.

The 256^3 single-subdomain workload (4,194,304 particles, one-cell halo,
gravity) and the same field cut into 8x8x8 periodic subdomains with a few
percent migrating per step: one fused step on the GPU against one whole
step of the CPU oracle on the same seeded input (the oracle runs in a few
seconds at this size).  Counts, ids and their order must match exactly;
positions and velocities to 1e-12; then the lock-step check: the oracle's
partition and append on the device's own post-advance records must give the
fused step's output bit for bit.  The same at full size for the nonlinear
drag law, the MAC-staggered field and migration after each RK2 stage (its
mid-step pool and send buffers too), each in its default launch shape.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import Case, compare_mid, compare_pools, lockstep_migration, say
from paper_2604_11008_amd import gen, pm

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name,shape", [("C2", (256, 4)), ("C2S", (256, 4)), ("C2", (512, 4))])
def test_full_size_step_matches_the_oracle(name, shape):
    say(f"[test] full-size {name} shape={shape}")
    c = Case(name, face=0.05, edge=0.01, corner=0.005)
    if name == "C2S":
        # keep dt/tau below 2 for the smallest tau at this resolution
        c.params.dt = min(c.dt, 0.015)
    pin = c.pin()
    send = c.send()
    pout = c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.set_tuning(*shape)
    ctx.step(c.field, c.dc, pin, pout, send, c.params)
    flags = ctx.get_status()
    say(f"  gpu flags {flags}")
    ref_out, ref_send, _, oflags = c.oracle_step(dt=c.params.dt)
    assert flags == oflags == 0
    delta = c.wl.L / c.wl.n
    compare_pools(send.to_host(), ref_send, c.dc.nsub * 27, c.wl.L, delta, what="send")
    ex, ev = compare_pools(pout.to_host(), ref_out, c.dc.nsub, c.wl.L, delta, what="out")
    say(f"  migrants {int(ref_send.count.sum())}; max rel err x {ex:.2e} v {ev:.2e}")
    lockstep_migration(c, ctx, pin, pout, send)
    say("  lock-step migration exact")


@pytest.mark.parametrize("name,drag,stagger", [("C2", "nonlinear", False),
                                               ("C2S", "stokes", True)])
def test_full_size_variant_matches_the_oracle(name, drag, stagger):
    say(f"[test] full-size {name} drag={drag} stagger={stagger}")
    c = Case(name, face=0.05, edge=0.01, corner=0.005, drag=drag, stagger=stagger)
    if name == "C2S":
        c.params.dt = min(c.dt, 0.015)
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.step(c.field, c.dc, pin, pout, send, c.params)
    flags = ctx.get_status()
    say(f"  gpu flags {flags}, shape {ctx.get_tuning()}")
    ref_out, ref_send, _, oflags = c.oracle_step(dt=c.params.dt)
    assert flags == oflags == 0
    delta = c.wl.L / c.wl.n
    compare_pools(send.to_host(), ref_send, c.dc.nsub * 27, c.wl.L, delta, what="send")
    ex, ev = compare_pools(pout.to_host(), ref_out, c.dc.nsub, c.wl.L, delta, what="out")
    say(f"  migrants {int(ref_send.count.sum())}; max rel err x {ex:.2e} v {ev:.2e}")


@pytest.mark.parametrize("name", ["C2", "C2S"])
def test_full_size_staged_step_matches_the_oracle(name):
    say(f"[test] full-size staged {name}")
    c = Case(name, face=0.05, edge=0.01, corner=0.005)
    if name == "C2S":
        c.params.dt = min(c.dt, 0.015)
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    mid = pm.DeviceStagePool.empty(c.host.base, c.host.cap, device=c.dev, size=pin.size)
    msend = pm.DeviceStagePool.empty(c.sb, c.sc, device=c.dev, size=send.size)
    ctx = c.ctx(pin, send)
    ctx.step_staged(c.field, c.dc, pin, mid, msend, pout, send, c.params)
    flags = ctx.get_status()
    say(f"  gpu flags {flags}, shape {ctx.get_tuning()}")
    rmid = gen.empty_stage_pool(c.host.base, c.host.cap)
    rms = gen.empty_stage_pool(c.sb, c.sc)
    rout, rsend = gen.empty_pool(c.host.base, c.host.cap), gen.empty_pool(c.sb, c.sc)
    oflags = oracle.step_staged(c.ofield, c.odc, c.params.dt, c.g, c.host, rmid, rms, rout,
                                rsend)
    assert flags == oflags == 0
    delta = c.wl.L / c.wl.n
    compare_mid(msend.to_host(), rms, c.dc.nsub * 27, c.wl.L, delta, "mid_send")
    compare_mid(mid.to_host(), rmid, c.dc.nsub, c.wl.L, delta, "mid")
    compare_pools(send.to_host(), rsend, c.dc.nsub * 27, c.wl.L, delta, what="send")
    ex, ev = compare_pools(pout.to_host(), rout, c.dc.nsub, c.wl.L, delta, what="out")
    say(f"  stage-1 migrants {int(rms.count.sum())}, stage-2 {int(rsend.count.sum())}; "
        f"max rel err x {ex:.2e} v {ev:.2e}")


@pytest.mark.parametrize("name", ["C3", "C4"])
def test_full_size_batched_workload_matches_the_oracle(name):
    """The 512^3 workloads at full size, field synthesised on the device like
    the benchmark's: blob-clustered 2^26 particles in 4x4x4 subdomains, and
    lognormal counts (about 8.2e7 particles) in 8x8x8: one fused step against
    one whole oracle step."""
    say(f"[test] full-size {name}")
    c = Case(name, face=0.05, edge=0.01, corner=0.005, slack=0.25, extra=4096,
             field_backend="device")
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.step(c.field, c.dc, pin, pout, send, c.params)
    flags = ctx.get_status()
    say(f"  gpu flags {flags}, shape {ctx.get_tuning()}")
    ref_out, ref_send, _, oflags = c.oracle_step()
    assert flags == oflags == 0
    delta = c.wl.L / c.wl.n
    compare_pools(send.to_host(), ref_send, c.dc.nsub * 27, c.wl.L, delta, what="send")
    ex, ev = compare_pools(pout.to_host(), ref_out, c.dc.nsub, c.wl.L, delta, what="out")
    say(f"  migrants {int(ref_send.count.sum())}; max rel err x {ex:.2e} v {ev:.2e}")
    # the same migration on the device's own post-advance positions, bit for
    # bit, so that exact parity does not rest on both sides rounding the
    # advance alike
    lockstep_migration(c, ctx, pin, pout, send)
    say("  lock-step migration exact")
