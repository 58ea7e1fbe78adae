"""Accuracy of the mixed-precision path against the FP64 oracle over many steps.

Mixed mode stores the field, velocities and tau in float32 and keeps
positions (and classification) in float64.  Workload: the 1024^3 recipe's
generator (blob-clustered particles, tau log-uniform in [0.01, 1], no
gravity, half a cell per step at the largest speed) on a 256^3 field, with
65,536 particles; the device advances them in place (interpolation + Heun
step) for 20 steps, the oracle does the same in float64 on the float64 field.
Both start from the same state: float64 positions, and velocities and tau as
float32 values.

Bound, with u = 2^-24 the float32 unit roundoff and |u|max the field's
largest component: each stage's interpolant is off by at most about 10 u
|u|max (storage of the 8 node values plus 7 lerps), and the Heun update adds
a few roundings of |V| <= |u|max; the drag factor dt/tau is below 1 here, so
the error in V grows at most by that much per step.  The tests allow
32 u |u|max per step.  Positions move by (dt/2)(V + V*) with dt |u|max at
most half a cell, so their error per step is at most the velocity error
times half a cell over |u|max, summed over the steps.

The nonlinear drag law multiplies the slip by f = 1 + 0.15 Re_p^0.687, evaluated
in float32 with a relative error of a few u; with dt f / tau below 1 the same
per-step allowance covers it.  The float64 path is held to the same check at
1e-12 per step.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import Case, say
from paper_2604_11008_amd import pm

pytestmark = pytest.mark.gpu

STEPS = 20
U32 = 2.0 ** -24


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _valid(pool):
    return np.concatenate([np.arange(int(b), int(b) + int(c))
                           for b, c in zip(pool.base, pool.count)])


@pytest.mark.parametrize("mode,drag", [("mixed", "stokes"), ("f64", "stokes"),
                                       ("mixed", "nonlinear"), ("f64", "nonlinear")])
def test_many_steps_against_the_fp64_oracle(mode, drag):
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
    per_step = 32 * U32 if mode == "mixed" else 1e-12
    errs = {}
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
            errs[k] = (ev, ex)
            say(f"  after {k:2d} step(s): max|dV|/|u|max {ev:.3e}  max|dX|/cell {ex:.3e}")
            assert ev <= k * per_step
            assert ex <= 0.5 * k * k * per_step + k * 1e-13
