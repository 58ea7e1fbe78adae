"""GPU parity of migration after each RK2 stage (the paper's scheme,
Sect. 3.2.2) against the oracle: the mid-step pool and its send buffers
(17 values per record) and the final pool, with bit-exact counts, ids and
order and values within 1e-12; the final state also matches the per-step
path up to periodic images and rounding."""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import Case, compare_mid, compare_pools, say
from paper_2604_11008_amd import gen, pm

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [("C1", None, None, None), ("C2", 40000, 32, None), ("C2S", 60000, 32, (4, 4, 4)),
         ("C3", 50000, 32, (4, 4, 4))]


@pytest.mark.parametrize("name,npart,n,p", CASES)
@pytest.mark.parametrize("drag", ["stokes", "nonlinear"])
def test_staged_step_matches_oracle(name, npart, n, p, drag):
    say(f"[test] staged step {name} {drag}")
    c = Case(name, npart, n, p, drag=drag, face=0.2, edge=0.05, corner=0.03)
    if name == "C2S":
        c.params.dt = min(c.dt, 0.015)
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    mid = pm.DeviceStagePool.empty(c.host.base, c.host.cap, device=c.dev, size=pin.size)
    msend = pm.DeviceStagePool.empty(c.sb, c.sc, device=c.dev, size=send.size)
    ctx = c.ctx(pin, send)
    ctx.step_staged(c.field, c.dc, pin, mid, msend, pout, send, c.params)
    flags = ctx.get_status()
    wg, items = ctx.get_tuning()[:2]
    assert wg == 256 and items <= 2  # the per-stage default, fewer for small pools
    rmid = gen.empty_stage_pool(c.host.base, c.host.cap)
    rms = gen.empty_stage_pool(c.sb, c.sc)
    rout, rsend = gen.empty_pool(c.host.base, c.host.cap), gen.empty_pool(c.sb, c.sc)
    oflags = oracle.step_staged(c.ofield, c.odc, c.params.dt, c.g, c.host, rmid, rms, rout,
                                rsend, drag=drag)
    assert flags == oflags == 0
    delta = c.wl.L / c.wl.n
    compare_mid(msend.to_host(), rms, c.dc.nsub * 27, c.wl.L, delta, "mid_send")
    compare_mid(mid.to_host(), rmid, c.dc.nsub, c.wl.L, delta, "mid")
    compare_pools(send.to_host(), rsend, c.dc.nsub * 27, c.wl.L, delta, what="send")
    ex, ev = compare_pools(pout.to_host(), rout, c.dc.nsub, c.wl.L, delta, what="out")
    say(f"  stage-1 migrants {int(rms.count.sum())}, stage-2 {int(rsend.count.sum())}; "
        f"max err x {ex:.2e} v {ev:.2e}")


# (wg, items[, blocks per CU, XCD-cyclic tile blocks])
@pytest.mark.parametrize("shape", [(256, 1), (256, 4), (512, 2), (256, 2, 0, 3)])
def test_staged_step_is_shape_invariant(shape):
    say(f"[test] staged shapes {shape}")
    c = Case("C2S", 60000, 32, (4, 4, 4), face=0.2, edge=0.05, corner=0.03)
    c.params.dt = min(c.dt, 0.015)
    outs = []
    for sh in [(256, 2), shape]:
        pin, send = c.pin(), c.send()
        pout = c.pout(pin.size)
        mid = pm.DeviceStagePool.empty(c.host.base, c.host.cap, device=c.dev, size=pin.size)
        msend = pm.DeviceStagePool.empty(c.sb, c.sc, device=c.dev, size=send.size)
        ctx = c.ctx(pin, send)
        ctx.set_tuning(*sh)
        ctx.step_staged(c.field, c.dc, pin, mid, msend, pout, send, c.params)
        assert ctx.get_status() == 0
        outs.append((pout.to_host(), mid.to_host()))
    for a, b in zip(outs[0], outs[1]):
        for name in ("x", "v", "id", "count"):
            np.testing.assert_array_equal(getattr(a, name), getattr(b, name))


def test_unbuilt_shape_and_mac_field_are_argument_errors():
    c = Case("C1", 2000, 16, (1, 1, 1))
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    mid = pm.DeviceStagePool.empty(c.host.base, c.host.cap, device=c.dev, size=pin.size)
    msend = pm.DeviceStagePool.empty(c.sb, c.sc, device=c.dev, size=send.size)
    ctx = c.ctx(pin, send)
    ctx.set_tuning(256, 8)
    with pytest.raises(pm.PMError, match="per-stage"):
        ctx.step_staged(c.field, c.dc, pin, mid, msend, pout, send, c.params)
    ctx.set_tuning(0, 0)
    mac = pm.DeviceField([u for u in c.field.u], c.wl.n, c.wl.halo, c.wl.L, device=c.dev,
                         stagger=True)
    with pytest.raises(pm.PMError, match="collocated"):
        ctx.step_staged(mac, c.dc, pin, mid, msend, pout, send, c.params)


def test_staged_graph_replays_match_eager():
    """pm_step_staged under pm_set_graph: every replay (two graphs, three
    replays each, eager torch work in between) equals the eager step."""
    say("[test] staged graph replays")
    c = Case("C2S", 40000, 32, (4, 4, 4), face=0.2, edge=0.05, corner=0.03)
    c.params.dt = min(c.dt, 0.015)
    pa, send = c.pin(), c.send()
    pb = c.pout(pa.size)
    mid = pm.DeviceStagePool.empty(c.host.base, c.host.cap, device=c.dev, size=pa.size)
    msend = pm.DeviceStagePool.empty(c.sb, c.sc, device=c.dev, size=send.size)
    ctx = c.ctx(pa, send)
    ea, eb = c.pin(), c.pout(pa.size)
    ref = []
    for _ in range(6):
        ctx.step_staged(c.field, c.dc, ea, mid, msend, eb, send, c.params)
        ea, eb = eb, ea
        ref.append(ea.to_host())
    assert ctx.get_status() == 0
    ctx.set_graph(True)
    for k in range(6):
        ctx.step_staged(c.field, c.dc, pa, mid, msend, pb, send, c.params)
        pa, pb = pb, pa
        torch.cuda.synchronize()
        _ = pa.x.sum().item()  # eager torch work between replays
        got = pa.to_host()
        np.testing.assert_array_equal(got.count, ref[k].count, err_msg=f"replay {k}")
        for q in range(c.dc.nsub):
            b, n = int(ref[k].base[q]), int(ref[k].count[q])
            for name in ("x", "v", "tau", "id"):
                np.testing.assert_array_equal(getattr(got, name)[..., b:b + n],
                                              getattr(ref[k], name)[..., b:b + n],
                                              err_msg=f"replay {k} {name} seg {q}")
    ctx.set_graph(False)
    assert ctx.get_status() == 0


def test_staged_mixed_precision_matches_the_per_step_path():
    """Mixed precision (FP32 field, velocities and tau; FP64 positions): the
    per-stage path runs the same Heun arithmetic as the per-step one, so the
    final velocities agree bit for bit and the positions up to the periodic
    image a stage-1 leaver is carried into (a few ulps of L)."""
    say("[test] staged mixed precision")
    c = Case("C2S", 60000, 32, (4, 4, 4), mode="mixed", face=0.2, edge=0.05, corner=0.03)
    c.params.dt = min(c.dt, 0.015)
    pin, send = c.pin(), c.send()
    ctx = c.ctx(pin, send)
    pout_a = c.pout(pin.size)
    ctx.step(c.field, c.dc, pin, pout_a, send, c.params)
    assert ctx.get_status() == 0
    a = pout_a.to_host()
    mid = pm.DeviceStagePool.empty(c.host.base, c.host.cap, vdtype=torch.float32,
                                   device=c.dev, size=pin.size)
    msend = pm.DeviceStagePool.empty(c.sb, c.sc, vdtype=torch.float32, device=c.dev,
                                     size=send.size)
    pout_b = c.pout(pin.size)
    ctx.step_staged(c.field, c.dc, pin, mid, msend, pout_b, send, c.params)
    assert ctx.get_status() == 0
    b = pout_b.to_host()

    def by_id(h):
        sel = np.concatenate([np.arange(int(s), int(s) + int(n))
                              for s, n in zip(h.base, h.count)])
        o = np.argsort(h.id[sel], kind="stable")
        return h.id[sel][o], h.x[:, sel][:, o], h.v[:, sel][:, o]

    ia, xa, va = by_id(a)
    ib, xb, vb = by_id(b)
    np.testing.assert_array_equal(ia, ib)
    np.testing.assert_array_equal(va, vb)
    dx = np.abs(xa - xb)
    dx = np.minimum(dx, np.abs(dx - c.wl.L))
    say(f"  stage-1 migrants {int(msend.count.sum().item())}; max |dx| {dx.max():.2e}")
    assert dx.max() <= 8 * np.spacing(c.wl.L)


def test_stage_one_overflow_counts_exactly_and_a_retry_succeeds():
    """mid_send buffers of one record: the stage-1 exchange flags
    SEND_OVERFLOW and still counts every leaver exactly (as the oracle
    does); `in` is intact, so a retry with regrown buffers gives the oracle's
    state."""
    say("[test] staged stage-1 overflow")
    c = Case("C2S", 40000, 32, (4, 4, 4), face=0.2, edge=0.05, corner=0.03)
    c.params.dt = min(c.dt, 0.015)
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    small = np.minimum(c.sc, 1)
    mid = pm.DeviceStagePool.empty(c.host.base, c.host.cap, device=c.dev, size=pin.size)
    msend = pm.DeviceStagePool.empty(c.sb, small, device=c.dev, size=send.size)
    ctx = c.ctx(pin, send)
    ctx.step_staged(c.field, c.dc, pin, mid, msend, pout, send, c.params)
    flags = ctx.get_status()
    say(f"  flags {pm.flag_names(flags)}")
    assert flags & pm.SEND_OVERFLOW
    rmid = gen.empty_stage_pool(c.host.base, c.host.cap)
    rms = gen.empty_stage_pool(c.sb, c.sc)
    rout, rsend = gen.empty_pool(c.host.base, c.host.cap), gen.empty_pool(c.sb, c.sc)
    oflags = oracle.step_staged(c.ofield, c.odc, c.params.dt, c.g, c.host, rmid, rms, rout,
                                rsend)
    assert oflags == 0
    np.testing.assert_array_equal(msend.to_host().count, rms.count)
    assert np.any(rms.count > small)  # some buffer held more than its one slot
    # regrow and retry from the intact input
    msend2 = pm.DeviceStagePool.empty(c.sb, c.sc, device=c.dev, size=send.size)
    send2 = c.send()
    ctx.step_staged(c.field, c.dc, pin, mid, msend2, pout, send2, c.params)
    assert ctx.get_status() == 0
    delta = c.wl.L / c.wl.n
    compare_mid(msend2.to_host(), rms, c.dc.nsub * 27, c.wl.L, delta, "mid_send")
    compare_pools(pout.to_host(), rout, c.dc.nsub, c.wl.L, delta, what="out")
