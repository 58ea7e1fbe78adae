"""GPU tests of the library's service entry points.

* pm_autotune: the tuned context gives bitwise the results of the default
  one; the cache file gets one line per problem key (grid, halo, precision,
  field arrangement, drag law, subdomains, pool extent, tile order), a second
  call on the same key reads it instead of timing, and another drag law is
  another key.
* pm_set_timing / pm_kernel_times: one record per eager step up to the limit.
* pm_touched_nodes (the byte accounting of the roofline): equal to an
  independent count of the distinct nodes of every particle's stage-1 (X)
  and stage-2 (X + dt V) stencils, for a periodic and a halo field.
"""
import numpy as np
import pytest
import torch

from gpu_cases import Case, assert_same_device_pools, say
from paper_2604_11008_amd import pm

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def c2s_case(drag="stokes"):
    c = Case("C2S", 60000, 32, (4, 4, 4), drag=drag)
    c.params = pm.Params(min(c.dt, 0.015), c.g, drag=drag)
    return c


def test_autotune_keeps_results_and_caches_by_problem(tmp_path):
    say("[test] autotune")
    c = c2s_case()
    pin = c.pin()
    send_a, out_a = c.send(), c.pout(pin.size)
    ref = c.ctx(pin, send_a)
    ref.step(c.field, c.dc, pin, out_a, send_a, c.params)
    assert ref.get_status() == 0

    cache = tmp_path / "tune.txt"
    ctx = c.ctx(pin, send_a)
    scratch_send, scratch_out = c.send(), c.pout(pin.size)
    ctx.autotune(c.field, c.dc, pin, scratch_out, scratch_send, c.params, cache_path=str(cache))
    tuned = ctx.get_tuning()
    say(f"  tuned {tuned}")
    assert (tuned[0], tuned[1]) in pm.SHAPES
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and "drag=0" in lines[0] and "stagger=0" in lines[0]
    assert f"wg={tuned[0]} items={tuned[1]} bpc={tuned[2]}" in lines[0]

    send_b, out_b = c.send(), c.pout(pin.size)
    ctx.step(c.field, c.dc, pin, out_b, send_b, c.params)
    assert ctx.get_status() == 0
    assert_same_device_pools(out_a, out_b, c.dc.nsub, "out after autotune")
    assert_same_device_pools(send_a, send_b, c.dc.nsub * 27, "send after autotune")

    # the same problem again: read from the cache, nothing appended
    ctx2 = c.ctx(pin, send_a)
    ctx2.autotune(c.field, c.dc, pin, scratch_out, scratch_send, c.params,
                  cache_path=str(cache))
    assert ctx2.get_tuning()[:3] == tuned[:3]
    assert len(cache.read_text().splitlines()) == 1

    # another drag law is another problem
    nl = pm.Params(c.params.dt, c.g, drag="nonlinear")
    ctx2.autotune(c.field, c.dc, pin, scratch_out, scratch_send, nl, cache_path=str(cache))
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and "drag=1" in lines[1]


def test_kernel_timing_records_each_step_up_to_the_limit():
    say("[test] kernel timing")
    c = c2s_case()
    pa, send = c.pin(), c.send()
    pb = c.pout(pa.size)
    ctx = c.ctx(pa, send)
    ctx.set_timing(4)
    for _ in range(6):
        ctx.step(c.field, c.dc, pa, pb, send, c.params)
        pa, pb = pb, pa
    assert ctx.get_status() == 0
    total, ms = ctx.kernel_times()
    say(f"  {len(ms)} records, total {total:.4f} ms")
    assert len(ms) == 4
    assert all(m > 0 for m in ms)
    assert total == pytest.approx(sum(ms), rel=1e-5)
    ctx.set_timing(0)
    total, ms = ctx.kernel_times()
    assert ms == [] and total == 0.0


def stencil_nodes(x, v, dt, n, L, halo):
    """Distinct linear node indices of the stage-1 and stage-2 stencils
    (nodes at cell centres; periodic wrap, or stored with a one-cell halo)."""
    S = n + 2 * halo
    xs = (x.astype(np.longdouble) + np.longdouble(dt) * v.astype(np.longdouble)).astype(
        np.float64)
    allnodes = []
    for X in (x, xs):
        c0 = []
        for a in range(3):
            i = np.floor(X[a] * (n / L) - 0.5).astype(np.int64)
            c0.append(i + 1 if halo else np.mod(i, n))
        for cz in (0, 1):
            for cy in (0, 1):
                for cx in (0, 1):
                    idx = []
                    for a, d in zip(range(3), (cx, cy, cz)):
                        j = c0[a] + d
                        idx.append(j if halo else np.mod(j, n))
                    allnodes.append(idx[0] + S * idx[1] + S * S * idx[2])
    return np.unique(np.concatenate(allnodes)).size


@pytest.mark.parametrize("name,npart,n,p", [("C1", None, None, None),
                                            ("C2", 40000, 32, None)])
def test_touched_nodes_match_an_independent_count(name, npart, n, p):
    say(f"[test] touched nodes {name}")
    c = Case(name, npart, n, p)
    pin = c.pin()
    ctx = c.ctx(pin, c.send())
    got = ctx.touched_nodes(c.field, pin, c.params)
    assert ctx.get_status() == 0
    h = c.host
    sel = np.concatenate([np.arange(int(b), int(b) + int(k)) for b, k in zip(h.base, h.count)])
    want = stencil_nodes(h.x[:, sel], h.v[:, sel].astype(np.float64), c.params.dt, c.wl.n,
                         c.wl.L, c.wl.halo)
    say(f"  touched {got} (independent count {want})")
    assert got == want
