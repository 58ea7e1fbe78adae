"""GPU tests of the cell re-sort (pm_sort), against its definition written
out with numpy: within every segment, records ordered by the cell key of
gen.cell_key (the canonical order's key) and, within a cell, by input
position; counts copied; records moved bit for bit.  A canonical pool is
its own re-sort; a shuffled one comes back in the canonical order's cells.
"""
import numpy as np
import pytest
import torch

from gpu_cases import Case, say
from paper_2604_11008_amd import gen, pm

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def expected(h, n, L):
    """Pool positions of each output record, segment by segment."""
    out = []
    for b, c in zip(h.base, h.count):
        b, c = int(b), int(c)
        x = h.x[:, b:b + c]
        cell = [np.clip(np.floor(x[a] * (n / L)).astype(np.int64), 0, n - 1) for a in range(3)]
        key = gen.cell_key(cell[0], cell[1], cell[2])
        out.append(b + np.lexsort((np.arange(c), key)))
    return out


def check(pin, pout, n, L, what):
    hi, ho = pin.to_host(), pout.to_host()
    np.testing.assert_array_equal(ho.count, hi.count, err_msg=f"{what} counts")
    for s, src in enumerate(expected(hi, n, L)):
        b, c = int(ho.base[s]), int(ho.count[s])
        for name in ("x", "v", "tau", "id"):
            np.testing.assert_array_equal(getattr(ho, name)[..., b:b + c],
                                          getattr(hi, name)[..., src],
                                          err_msg=f"{what} {name} seg {s}")


@pytest.mark.parametrize("name,npart,n,p,order,mode", [
    ("C2S", 60000, 32, (4, 4, 4), "shuffled", None),
    ("C2S", 60000, 32, (4, 4, 4), "canonical", None),
    ("C1", None, None, None, "shuffled", "mixed"),
    ("C2", 70000, 64, None, "shuffled", None),
    ("C3", 90000, 64, (4, 4, 4), "rowmajor", None),
])
def test_sort_matches_its_definition(name, npart, n, p, order, mode):
    say(f"[test] re-sort {name} {order} {mode}")
    c = Case(name, npart, n, p, order=order, mode=mode)
    pin, send = c.pin(), c.send()
    pout = c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.sort(c.field, pin, pout)
    assert ctx.get_status() == 0
    check(pin, pout, c.wl.n, c.wl.L, f"{name} {order}")
    if order == "canonical":
        h, o = pin.to_host(), pout.to_host()
        np.testing.assert_array_equal(o.id, h.id)


def test_sorted_pool_steps_like_the_unsorted_one():
    """The step does not depend on the order within a segment beyond the
    order of its output: the same particles, positions and velocities."""
    say("[test] step after re-sort")
    c = Case("C2S", 60000, 32, (4, 4, 4), order="shuffled")
    c.params = pm.Params(min(c.dt, 0.015), c.g)
    pin, send = c.pin(), c.send()
    ps, pa, pb = c.pout(pin.size), c.pout(pin.size), c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.sort(c.field, pin, ps)
    ctx.step(c.field, c.dc, pin, pa, send, c.params)
    send2 = c.send()
    ctx.step(c.field, c.dc, ps, pb, send2, c.params)
    assert ctx.get_status() == 0
    a, b = pa.to_host(), pb.to_host()
    np.testing.assert_array_equal(a.count, b.count)
    for s in range(c.dc.nsub):
        lo, k = int(a.base[s]), int(a.count[s])
        oa = np.argsort(a.id[lo:lo + k])
        ob = np.argsort(b.id[lo:lo + k])
        np.testing.assert_array_equal(a.id[lo:lo + k][oa], b.id[lo:lo + k][ob])
        np.testing.assert_array_equal(a.x[:, lo:lo + k][:, oa], b.x[:, lo:lo + k][:, ob])
        np.testing.assert_array_equal(a.v[:, lo:lo + k][:, oa], b.v[:, lo:lo + k][:, ob])


def test_sort_errors_and_overflow():
    """The same pool as input and output is an argument error; an output
    segment smaller than its count gets PM_F_DEST_OVERFLOW, the exact count,
    and the records that fit (the first ones in sorted order)."""
    say("[test] re-sort errors")
    c = Case("C2S", 60000, 32, (4, 4, 4), order="shuffled")
    pin, send = c.pin(), c.send()
    ctx = c.ctx(pin, send)
    with pytest.raises(pm.PMError, match="different"):
        ctx.sort(c.field, pin, pin)
    small_cap = np.maximum(c.host.count - 5, 0)
    pout = pm.DevicePool.empty(c.host.base, small_cap, device=c.dev, size=pin.size)
    ctx.sort(c.field, pin, pout)
    flags = ctx.get_status()
    assert flags == pm.DEST_OVERFLOW, pm.flag_names(flags)
    hi, ho = pin.to_host(), pout.to_host()
    np.testing.assert_array_equal(ho.count, hi.count)
    for s, src in enumerate(expected(hi, c.wl.n, c.wl.L)):
        b, k = int(ho.base[s]), int(small_cap[s])
        np.testing.assert_array_equal(ho.id[b:b + k], hi.id[src[:k]])
