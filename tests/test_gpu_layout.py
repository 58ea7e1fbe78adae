"""GPU: a field stored node-interleaved (the three components of a node next
to each other) gives bitwise the results of the same field stored as one
array per component, through every entry point that interpolates (Sect.
2.2), per-stage migration included (Sect. 3.2.2), and so the oracle's; the
layout's argument checks.

The interleaved copy is made by stacking the split arrays: a change of
storage only, no arithmetic.
"""
import math
import types

import numpy as np
import pytest
import torch

import oracle
from gpu_cases import Case, assert_same_device_pools, compare_pools, say
from paper_2604_11008_amd import gen, pm

pytestmark = pytest.mark.gpu

TWO_PI = 2 * math.pi


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def interleaved(field):
    """The same field, node-interleaved (component fastest)."""
    return pm.DeviceField(torch.stack(field.u, dim=1), field.n, field.halo, field.L,
                          device=field.u[0].device, interleaved=True)


@pytest.mark.parametrize("halo,mixed", [(0, False), (1, False), (0, True), (1, True)])
def test_interleaved_interp_is_bitwise_the_split_interp(halo, mixed):
    """Positions everywhere in the box, periodic images included (the x
    corner n-1 pairs with node 0), and the box's edges."""
    say(f"[test] interleaved interp halo={halo} mixed={mixed}")
    n = 40
    u = gen.spectral_field(n, 4, 8, gen.seeds(0)[0])
    stored = [gen.with_halo(c) if halo else c for c in u]
    if mixed:
        stored = [np.asarray(c, dtype=np.float32) for c in stored]
    rng = np.random.default_rng(11)
    lo, hi = (0.0, TWO_PI) if halo else (-TWO_PI + TWO_PI / n, 2 * TWO_PI - 0.2)
    X = rng.uniform(lo, hi, (3, 20011))
    X[:, :5] = [[0.0, TWO_PI * (1 - 1e-16), 0.5 * TWO_PI / n, TWO_PI * (1 - 0.4 / n), 3.0]] * 3
    dev = torch.device("cuda:0")
    fs = pm.DeviceField(stored, n, halo, TWO_PI, device=dev)
    fi = interleaved(fs)
    ctx = pm.Context(1, 1, 1, device=dev)
    Xd = torch.from_numpy(X).to(dev)
    a = ctx.interp(fs, Xd).cpu().numpy()
    b = ctx.interp(fi, Xd).cpu().numpy()
    assert ctx.get_status() == 0
    np.testing.assert_array_equal(a, b)
    if not mixed:
        ref, f0 = oracle.interp(oracle.Field(stored, n, halo, TWO_PI), X)
        assert f0 == 0
        err = np.abs(b - ref).max() / max(1.0, np.abs(ref).max())
        say(f"  bitwise equal; max rel err vs oracle {err:.2e}")
        assert err <= 1e-12


STEP_CASES = [
    ("C1", None, None, None, "f64", "stokes"),
    ("C2", 40000, 32, None, "f64", "stokes"),
    ("C2", 40000, 32, None, "mixed", "nonlinear"),
    ("C2S", 60000, 32, (4, 4, 4), "mixed", "stokes"),
    ("C3", 50000, 32, (4, 4, 4), "f64", "nonlinear"),
]


@pytest.mark.parametrize("name,npart,n,p,mode,drag", STEP_CASES)
def test_interleaved_step_is_bitwise_the_split_step(name, npart, n, p, mode, drag):
    """pm_step in three launch shapes, and the plain path's pm_interp_advance,
    on periodic and halo fields, both drag laws and both precisions."""
    say(f"[test] interleaved step {name} {mode} {drag}")
    c = Case(name, npart, n, p, mode=mode, drag=drag)
    if name == "C2S":
        c.params = pm.Params(min(c.dt, 0.015), c.g, drag=drag)
    fi = interleaved(c.field)
    pin = c.pin()
    ctx = c.ctx(pin, c.send())
    for wg, items in ((256, 1), (256, 4), (512, 2)):
        say(f"  shape {wg}x{items}")
        ctx.set_tuning(wg, items)
        res = []
        for f in (c.field, fi):
            send, out = c.send(), c.pout(pin.size)
            ctx.step(f, c.dc, pin, out, send, c.params)
            assert ctx.get_status() == 0
            res.append((out, send))
        assert_same_device_pools(res[0][0], res[1][0], c.dc.nsub, f"out {wg}x{items}")
        assert_same_device_pools(res[0][1], res[1][1], c.dc.nsub * 27, f"send {wg}x{items}")
    adv = []
    for f in (c.field, fi):
        pa = c.pin()
        ctx.interp_advance(f, pa, c.params)
        assert ctx.get_status() == 0
        adv.append(pa)
    assert_same_device_pools(adv[0], adv[1], c.dc.nsub, "interp_advance")


def test_interleaved_step_matches_the_oracle():
    say("[test] interleaved step vs oracle C3")
    c = Case("C3", 50000, 32, (4, 4, 4))
    fi = interleaved(c.field)
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.step(fi, c.dc, pin, pout, send, c.params)
    flags = ctx.get_status()
    ref_out, ref_send, _, oflags = c.oracle_step()
    assert flags == oflags == 0
    delta = c.wl.L / c.wl.n
    compare_pools(send.to_host(), ref_send, c.dc.nsub * 27, c.wl.L, delta, what="send")
    ex, ev = compare_pools(pout.to_host(), ref_out, c.dc.nsub, c.wl.L, delta, what="out")
    say(f"  migrants {int(ref_send.count.sum())}; max err x {ex:.2e} v {ev:.2e}")


@pytest.mark.parametrize("mode,shape", [("f64", (256, 4)), ("mixed", (256, 2)),
                                        ("mixed", (256, 4))])
def test_interleaved_step_in_the_timed_shape(mode, shape):
    """The 1024^3 workload's recipe at 256^3 (2^22 blob-clustered particles,
    8x8x8 subdomains) in the launch shapes its interleaved runs are timed in
    (256 x 4 at FP64, 256 x 2 mixed) and the split runs' 256 x 4, three steps
    in a row: bitwise the split layout's pools after each."""
    say(f"[test] interleaved timed shape {mode} {shape}, 256^3, 2^22 particles")
    c = Case("C5", npart=1 << 22, n=256, mode=mode, face=0.05, edge=0.01, corner=0.005)
    fi = interleaved(c.field)
    pa = [c.pin(), c.pin()]
    pb = [c.pout(pa[0].size), c.pout(pa[0].size)]
    ctx = c.ctx(pa[0], c.send())
    ctx.set_tuning(*shape)
    for k in range(3):
        sends = []
        for j, f in enumerate((c.field, fi)):
            send = c.send()
            ctx.step(f, c.dc, pa[j], pb[j], send, c.params)
            sends.append(send)
            pa[j], pb[j] = pb[j], pa[j]
        assert ctx.get_status() == 0
        assert_same_device_pools(pa[0], pa[1], c.dc.nsub, f"out step {k + 1}")
        assert_same_device_pools(sends[0], sends[1], c.dc.nsub * 27, f"send step {k + 1}")
        say(f"  step {k + 1}: bitwise equal")


STAGED_CASES = [
    ("C2", 40000, 32, None, "f64", "stokes", (256, 2)),
    ("C2S", 60000, 32, (4, 4, 4), "f64", "nonlinear", (256, 4)),
    ("C2S", 60000, 32, (4, 4, 4), "mixed", "stokes", (512, 2)),
    ("C3", 50000, 32, (4, 4, 4), "mixed", "nonlinear", (256, 1)),
]


@pytest.mark.parametrize("name,npart,n,p,mode,drag,shape", STAGED_CASES)
def test_interleaved_staged_step_is_bitwise_the_split_step(name, npart, n, p, mode, drag,
                                                           shape):
    """Migration after each RK2 stage (Sect. 3.2.2): the mid-step pool and
    buffers and the final pool and buffers, bit for bit."""
    say(f"[test] interleaved staged step {name} {mode} {drag} {shape}")
    c = Case(name, npart, n, p, mode=mode, drag=drag, face=0.2, edge=0.05, corner=0.03)
    c.params = pm.Params(min(c.dt, 0.015), c.g, drag=drag)
    fi = interleaved(c.field)
    res = []
    for f in (c.field, fi):
        pin, send = c.pin(), c.send()
        pout = c.pout(pin.size)
        mid = pm.DeviceStagePool.empty(c.host.base, c.host.cap, vdtype=c.vdt, device=c.dev,
                                       size=pin.size)
        msend = pm.DeviceStagePool.empty(c.sb, c.sc, vdtype=c.vdt, device=c.dev,
                                         size=send.size)
        ctx = c.ctx(pin, send)
        ctx.set_tuning(*shape)
        ctx.step_staged(f, c.dc, pin, mid, msend, pout, send, c.params)
        assert ctx.get_status() == 0
        res.append((pout, send, mid.to_host(), msend.to_host()))
    assert_same_device_pools(res[0][0], res[1][0], c.dc.nsub, "out")
    assert_same_device_pools(res[0][1], res[1][1], c.dc.nsub * 27, "send")
    for k in (2, 3):
        for name_ in ("x", "v", "xs", "vs", "a", "tau", "id", "count"):
            np.testing.assert_array_equal(getattr(res[0][k], name_), getattr(res[1][k], name_),
                                          err_msg=f"mid {name_}")


@pytest.mark.parametrize("halo,kind", [(0, "f64"), (1, "f64"), (0, "f32"), (1, "f32"),
                                       (0, "f64->f32"), (1, "f64->f32")])
def test_library_interleave_copies_the_field(halo, kind):
    """pm_field_interleave writes exactly the stacked components (a copy, or
    from float64 the float32 values a cast gives), and a step on its output
    is bitwise the split step on the same values."""
    say(f"[test] pm_field_interleave halo={halo} {kind}")
    c = Case("C2" if halo else "C1", 30000, 24, None if halo else (2, 2, 2),
             mode="f64" if kind == "f64" else "mixed")
    assert c.wl.halo == halo
    if kind == "f64->f32":
        src = pm.DeviceField(c.fh, c.wl.n, c.wl.halo, c.wl.L, device=c.dev)
        fi = pm.interleave_field(src, dtype=torch.float32)
    else:
        fi = pm.interleave_field(c.field)
    torch.cuda.synchronize()
    ref = torch.stack(c.field.u, dim=1).reshape(-1)
    assert torch.equal(fi.u[0], ref)
    # again into the same buffer, after spoiling it
    fi.u[0].fill_(float("nan"))
    if kind == "f64->f32":
        pm.interleave_field(src, out=fi.u[0], dtype=torch.float32)
    else:
        pm.interleave_field(c.field, out=fi.u[0])
    torch.cuda.synchronize()
    assert torch.equal(fi.u[0], ref)
    with pytest.raises(pm.PMError):
        pm.interleave_field(c.field, out=fi.u[0][:-1])
    pin = c.pin()
    ctx = c.ctx(pin, c.send())
    res = []
    for f in (c.field, fi):
        send, out = c.send(), c.pout(pin.size)
        ctx.step(f, c.dc, pin, out, send, c.params)
        assert ctx.get_status() == 0
        res.append((out, send))
    assert_same_device_pools(res[0][0], res[1][0], c.dc.nsub, "out")
    assert_same_device_pools(res[0][1], res[1][1], c.dc.nsub * 27, "send")


def test_autotune_and_noalloc_on_an_interleaved_field():
    say("[test] interleaved autotune and noalloc, C2")
    c = Case("C2", 40000, 32, None)
    fi = interleaved(c.field)
    pin = c.pin()
    send_a, out_a = c.send(), c.pout(pin.size)
    ctx = c.ctx(pin, send_a)
    ctx.step(c.field, c.dc, pin, out_a, send_a, c.params)
    assert ctx.get_status() == 0
    send_b, out_b = c.send(), c.pout(pin.size)
    ctx.autotune(fi, c.dc, pin, out_b, send_b, c.params)
    assert ctx.get_status() == 0
    ctx.step(fi, c.dc, pin, out_b, send_b, c.params)
    assert ctx.get_status() == 0
    assert_same_device_pools(out_a, out_b, c.dc.nsub, "autotuned out")
    send_c, out_c = c.send(), c.pout(pin.size)
    flags = torch.full((1,), -1, dtype=torch.int32, device=c.dev)
    pm.step_noalloc(fi, c.dc, pin, out_c, send_c, c.params, flags)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0
    assert_same_device_pools(out_a, out_c, c.dc.nsub, "noalloc out")
    assert_same_device_pools(send_a, send_c, c.dc.nsub * 27, "noalloc send")


def test_interleaved_layout_argument_errors():
    """Rejected before any launch: an unknown layout, an interleaved MAC
    field, u[1] or u[2] set on an interleaved field; a binding-built field of
    the wrong size."""
    say("[test] interleaved layout argument errors")
    c = Case("C1")
    fi = interleaved(c.field)
    pin = c.pin()
    send, out = c.send(), c.pout(pin.size)
    ctx = c.ctx(pin, send)

    def raw(**kw):
        f = pm._Field.from_buffer_copy(fi.c)
        for k, v in kw.items():
            if k == "u":
                for a in range(3):
                    f.u[a] = v[a]
            else:
                setattr(f, k, v)
        return types.SimpleNamespace(c=f)

    bad = [
        (raw(layout=2), b"layout"),
        (raw(stagger=1), b"collocated"),
        (raw(u=[fi.c.u[0], fi.c.u[0], None]), b"NULL for an interleaved"),
        (raw(u=[None, None, None]), b"u[0] is NULL"),
    ]
    for f, msg in bad:
        with pytest.raises(pm.PMError):
            ctx.step(f, c.dc, pin, out, send, c.params)
        assert msg in pm.lib().pm_last_error(), pm.lib().pm_last_error()
    # the step is untouched by the rejected calls
    ctx.step(fi, c.dc, pin, out, send, c.params)
    assert ctx.get_status() == 0
    with pytest.raises(pm.PMError):
        pm.DeviceField(fi.u[0][:-3], fi.n, fi.halo, fi.L, device=c.dev, interleaved=True)
    with pytest.raises(pm.PMError):
        pm.DeviceField(fi.u[0], fi.n, fi.halo, fi.L, device=c.dev, interleaved=True,
                       stagger=True)


def test_geometry_calls_take_an_interleaved_field():
    """pm_touched_nodes and pm_sort read only the field's grid: the same
    count and the same re-sorted pool from either layout."""
    say("[test] touched nodes and re-sort on an interleaved field")
    c = Case("C3", 50000, 32, (4, 4, 4), order="shuffled")
    fi = interleaved(c.field)
    pin = c.pin()
    ctx = c.ctx(pin, c.send())
    ta = ctx.touched_nodes(c.field, pin, c.params)
    tb = ctx.touched_nodes(fi, pin, c.params)
    assert ta == tb > 0
    outs = []
    for f in (c.field, fi):
        out = c.pout(pin.size)
        ctx.sort(f, pin, out)
        assert ctx.get_status() == 0
        outs.append(out)
    assert_same_device_pools(outs[0], outs[1], c.dc.nsub, "sorted")
