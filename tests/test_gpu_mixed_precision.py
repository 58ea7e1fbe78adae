"""Accuracy of the mixed-precision path against the FP64 oracle.

Mixed mode stores the field, velocities and tau in float32 and keeps
positions (and classification) in float64.  The oracle runs the same steps
in float64 on the float64 field, from the same start state: float64
positions, and velocities and tau as the float32 values the device holds.

Bars (velocities over |u|max, the field's largest component; positions in
cells, periodic images folded), the same for every test here:

  after 1 step:   |dV| <= 1e-6,  |dX| <= 2e-8 cell
  after 20 steps: |dV| <= 4e-6,  |dX| <= 1e-5 cell

The velocity bars are the analytic estimate made before any kernel existed:
each stage's interpolant carries the float32 rounding of the 8 node values
and 7 lerps (a few u |u|max, u = 2^-24 = 6e-8), the Heun update a few more
roundings of |V| <= |u|max, and with dt/tau below 1 they do not grow by more
than that per step; over many steps they add up more like a random walk
than linearly.  Positions move by (dt/2)(V + V*) with dt |u|max at most half
a cell: after one step only the stage-1 velocity V* = V + dt A1 carries an
error, (dt/tau) times the interpolation error, so |dX| is about a quarter of
a cell times h |dU| (h = dt/tau <= 0.22): below 1e-8 cell; after k steps
|dX| <= (1/2) sum_j |dV_j| / |u|max cells, below 1e-5 cell with the
velocity bar.  Measured (the 1024^3 workload, 2^20 lowest ids): |dV| 4.3e-8
and 2.9e-7, |dX| 7e-10 and 1.5e-6 cell -- margins of 14x or more on the
velocities and 7x or more on the positions.

The nonlinear drag law multiplies the slip by f = 1 + 0.15 Re_p^0.687, evaluated
in float32 with a relative error of a few u; the same bars apply.  The float64
path is held to 1e-12 per step.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import Case, lockstep_migration, per_id_errors, say
from paper_2604_11008_amd import gen, pm

pytestmark = pytest.mark.gpu

STEPS = 20
V_BAR = {1: 1e-6, STEPS: 4e-6}
X_BAR = {1: 2e-8, STEPS: 1e-5}


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _valid(pool):
    return np.concatenate([np.arange(int(b), int(b) + int(c))
                           for b, c in zip(pool.base, pool.count)])


def _bars(mode, k):
    if mode == "mixed":
        return V_BAR[k], X_BAR[k]
    return k * 1e-12, 0.5 * k * k * 1e-12 + k * 1e-13


@pytest.mark.parametrize("mode,drag", [("mixed", "stokes"), ("f64", "stokes"),
                                       ("mixed", "nonlinear"), ("f64", "nonlinear")])
def test_many_steps_against_the_fp64_oracle(mode, drag):
    """The in-place advance (interpolation + Heun) of 65,536 particles of the
    1024^3 recipe on a 256^3 field, 20 steps, against the oracle's."""
    say(f"[test] {STEPS} steps, mode {mode}, drag {drag}, 256^3, 65536 particles")
    c = Case("C5", npart=1 << 16, n=256, mode=mode, drag=drag)
    umax = max(float(np.abs(u).max()) for u in c.fh)
    delta = c.wl.L / c.wl.n
    assert c.dt * umax <= 0.5 * delta * (1 + 1e-12)
    assert c.dt / float(np.min(c.host.tau[_valid(c.host)])) < 1.0

    idx = _valid(c.host)
    x = c.host.x[:, idx].astype(np.float64)
    v = c.host.v[:, idx].astype(np.float64)
    tau = c.host.tau[idx].astype(np.float64)

    pin = c.pin()
    ctx = pm.Context(pin.size, 1, c.dc.nsub, device=c.dev)
    tidx = torch.as_tensor(idx, device=c.dev)
    for k in range(1, STEPS + 1):
        ctx.interp_advance(c.field, pin, c.params)
        x, v, oflags = oracle.advance(c.ofield, x, v, tau, c.dt, c.g, drag=drag,
                                      nu=c.params.nu, density_ratio=c.params.density_ratio)
        assert oflags == 0
        if k in (1, STEPS):
            assert ctx.get_status() == 0
            gx = pin.x[:, tidx].cpu().numpy()
            gv = pin.v[:, tidx].double().cpu().numpy()
            ev = float(np.abs(gv - v).max()) / umax
            ex = float(np.abs(gx - x).max()) / delta
            say(f"  after {k:2d} step(s): max|dV|/|u|max {ev:.3e}  max|dX|/cell {ex:.3e}")
            vb, xb = _bars(mode, k)
            assert ev <= vb and ex <= xb, (ev, vb, ex, xb)


@pytest.mark.parametrize("shape", [(256, 4), (256, 2)])
def test_mixed_fused_step_in_the_timed_shapes(shape):
    """The fused mixed-precision kernel in the launch shapes the 1024^3
    workload is timed in (1024- and 512-record tiles), on its recipe at
    256^3 with 4,194,304 blob-clustered particles in 8x8x8 subdomains (8
    tiles per segment on average, up to several tens): one step against the
    FP64 oracle per id within the mixed bars, then the migration lock-step
    against the oracle's partition and append on the device's own
    post-advance records, bit for bit."""
    say(f"[test] mixed fused step, shape {shape}, 256^3, 2^22 particles, 8x8x8")
    c = Case("C5", npart=1 << 22, n=256, mode="mixed", face=0.05, edge=0.01, corner=0.005)
    umax = max(float(np.abs(u).max()) for u in c.fh)
    tiles = np.ceil(c.host.count / (shape[0] * shape[1]))
    say(f"  tiles per segment: mean {tiles.mean():.1f}, max {int(tiles.max())}")
    assert tiles.max() >= 8
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.set_tuning(*shape)
    ctx.step(c.field, c.dc, pin, pout, send, c.params)
    assert ctx.get_status() == 0
    assert tuple(ctx.get_tuning()[:2]) == shape
    ref_out, ref_send, _, oflags = c.oracle_step()
    assert oflags == 0
    got = pout.to_host()
    delta = c.wl.L / c.wl.n
    ev, ex = per_id_errors(got, ref_out, c.wl.L, delta, umax)
    # ownership can differ from the FP64 oracle's only for a particle within
    # about 1e-9 cell of a subdomain face: none is expected at this size
    owners_differ = int(np.abs(got.count - ref_out.count).sum())
    say(f"  vs FP64 oracle: max|dV|/|u|max {ev:.3e}, max|dX|/cell {ex:.3e}, "
        f"count differences {owners_differ}")
    assert ev <= V_BAR[1] and ex <= X_BAR[1]
    assert owners_differ <= 2
    migrants = lockstep_migration(c, ctx, pin, pout, send)
    say(f"  lock-step migration exact ({migrants} migrants)")


def _sample(p, nmax):
    """Records of device pool p with id < nmax, in pool order, on the host
    (x float64; v and tau as stored) with the number in each segment."""
    size = p.x.shape[1]
    valid = torch.zeros(size, dtype=torch.bool, device=p.x.device)
    base, count = p.base.cpu().numpy(), p.count.cpu().numpy()
    for b, n in zip(base, count):
        if n > 0:
            valid[int(b):int(b) + int(n)] = True
    keep = valid & (p.id < nmax)
    sel = torch.nonzero(keep).squeeze(1)
    seg = torch.bucketize(sel, torch.as_tensor(base, device=sel.device), right=True) - 1
    counts = torch.bincount(seg, minlength=len(base)).cpu().numpy().astype(np.int64)
    return (p.x[:, sel].cpu().numpy(), p.v[:, sel].cpu().numpy(), p.tau[sel].cpu().numpy(),
            p.id[sel].cpu().numpy().astype(np.uint64), counts)


def _host_pool(sample, vdtype):
    x, v, tau, ids, counts = sample
    base, cap = gen.layout(counts, slack=0.5, extra=256)
    pool = gen.empty_pool(base, cap, vdtype)
    start = 0
    for q, n in enumerate(counts):
        b = int(base[q])
        pool.x[:, b:b + n] = x[:, start:start + n]
        pool.v[:, b:b + n] = v[:, start:start + n]
        pool.tau[b:b + n] = tau[start:start + n]
        pool.id[b:b + n] = ids[start:start + n]
        start += n
    pool.count[:] = counts
    return pool


@pytest.mark.slow
def test_full_size_1024_mixed_against_the_fp64_oracle():
    """The 1024^3 workload at full size (2^28 blob-clustered particles, FP32
    field, 8x8x8 subdomains) in the launch shape its benchmark times: 20
    fused steps on the device; the oracle follows the 2^20 lowest ids from
    the same start state in FP64 on the float64 field, whole steps with the
    same decomposition (particles do not interact, so the subsample evolves
    as in the whole pool).  Errors per id after the first and the last step
    within the mixed bars."""
    nmax = 1 << 20
    say("[test] full-size 1024^3 mixed, 2^28 particles, 20 steps, 2^20 lowest ids")
    c = Case("C5", mode="mixed", face=0.05, edge=0.01, corner=0.005, slack=0.25,
             extra=4096, field_backend="device")
    umax = max(float(np.abs(u).max()) for u in c.fh)
    delta = c.wl.L / c.wl.n
    pa, send = c.pin(), c.send()
    pb = c.pout(pa.size)
    ctx = c.ctx(pa, send)
    start = _sample(pa, nmax)
    got = {}
    for k in range(1, STEPS + 1):
        ctx.step(c.field, c.dc, pa, pb, send, c.params)
        pa, pb = pb, pa
        if k in (1, STEPS):
            got[k] = _sample(pa, nmax)
    assert ctx.get_status() == 0
    assert tuple(ctx.get_tuning()[:2]) == (256, 4)
    del pa, pb, send
    # the oracle's state is float64 throughout (the float32 start values
    # promoted exactly)
    host = _host_pool(start, np.float64)
    osb, osc = gen.send_layout(host.count, face=0.2, edge=0.05, corner=0.03)
    for k in range(1, STEPS + 1):
        nxt = gen.empty_pool(host.base, host.cap, np.float64)
        _, fl = oracle.step(c.ofield, c.odc, c.dt, c.g, host, nxt, gen.empty_pool(osb, osc))
        assert fl == 0
        host = nxt
        if k in got:
            ev, ex = per_id_errors(_host_pool(got[k], np.float32), host, c.wl.L, delta, umax)
            say(f"  after {k:2d} step(s): max|dV|/|u|max {ev:.3e}  max|dX|/cell {ex:.3e}")
            assert ev <= V_BAR[k] and ex <= X_BAR[k], (k, ev, ex)
