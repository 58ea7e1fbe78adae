"""GPU parity: the HIP library, called through its C ABI, against the CPU
oracle on the same seeded inputs.

Interpolation and drag: within 1e-12 (float64); classification, scan, pack,
compaction and append: bit-exact, on identical positions.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_cases import Case, assert_same_device_pools, compare_pools, say, seg
from paper_2604_11008_amd import gen, pm

pytestmark = pytest.mark.gpu

TWO_PI = 2 * math.pi


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# ---------------------------------------------------------------------------
# interpolation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("halo", [0, 1])
def test_interp_matches_oracle(halo):
    say(f"[test] interp halo={halo}")
    n = 48
    u = gen.spectral_field(n, 4, 8, gen.seeds(0)[0])
    stored = [gen.with_halo(c) if halo else c for c in u]
    of = oracle.Field(stored, n, halo, TWO_PI)
    rng = np.random.default_rng(7)
    lo, hi = (0.0, TWO_PI) if halo else (-TWO_PI + TWO_PI / n, 2 * TWO_PI - 0.2)
    X = rng.uniform(lo, hi, (3, 30011))
    X[:, :6] = [[0.0, TWO_PI * (1 - 1e-16), 0.5 * TWO_PI / n, 1e-300, 3.0, 1.0]] * 3
    ref, f0 = oracle.interp(of, X)
    dev = torch.device("cuda:0")
    field = pm.DeviceField(stored, n, halo, TWO_PI, device=dev)
    ctx = pm.Context(1, 1, 1, device=dev)
    got = ctx.interp(field, torch.from_numpy(X).to(dev)).cpu().numpy()
    assert ctx.get_status() == f0 == 0
    err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
    say(f"  max rel err {err:.2e}")
    assert err <= 1e-12


def test_interp_reproduces_a_trilinear_field_bit_exactly():
    say("[test] interp trilinear exact")
    N, L = 64, 64.0
    coefs = [(3, 2, -1, 1, 1, 0, -2, 1), (-5, 1, 4, -3, 0, 2, 1, -1), (7, -2, 0, 5, -1, 1, 0, 2)]

    def analytic(c, x, y, z):
        a, b, cc, d, e, f, g, h = c
        return a + b * x + cc * y + d * z + e * x * y + f * y * z + g * x * z + h * x * y * z

    idx = np.arange(-1, N + 1) + 0.5
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    stored = [analytic(c, x, y, z).reshape(-1) for c in coefs]
    X = np.round(np.random.default_rng(3).uniform(0, L - 1 / 64, (3, 5000)) * 64) / 64
    dev = torch.device("cuda:0")
    field = pm.DeviceField(stored, N, 1, L, device=dev)
    ctx = pm.Context(1, 1, 1, device=dev)
    got = ctx.interp(field, torch.from_numpy(X).to(dev)).cpu().numpy()
    for c in range(3):
        np.testing.assert_array_equal(got[c], analytic(coefs[c], *X))


# ---------------------------------------------------------------------------
# advance
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,npart,n,p", [("C1", 20000, 32, (2, 2, 2)),
                                            ("C2", 30000, 32, (1, 1, 1))])
def test_interp_advance_matches_oracle(name, npart, n, p):
    say(f"[test] interp_advance {name}")
    c = Case(name, npart, n, p)
    pin = c.pin()
    send = c.send()
    ctx = c.ctx(pin, send)
    ctx.interp_advance(c.field, pin, c.params)
    assert ctx.get_status() == 0
    got = pin.to_host()
    for q in range(c.dc.nsub):
        s = seg(c.host, q)
        xr, vr, _ = oracle.advance(c.ofield, c.host.x[:, s], c.host.v[:, s], c.host.tau[s],
                                   c.dt, c.g)
        ex = np.abs(got.x[:, s] - xr) / np.maximum(np.abs(xr), c.wl.L / c.wl.n)
        ev = np.abs(got.v[:, s] - vr) / max(1.0, np.abs(vr).max())
        assert ex.max() <= 1e-12 and ev.max() <= 1e-12, (ex.max(), ev.max())
        np.testing.assert_array_equal(got.id[s], c.host.id[s])


# ---------------------------------------------------------------------------
# migration on identical positions: bit-exact
# ---------------------------------------------------------------------------

def special_positions(rng, p, n):
    """Positions near faces, on faces, across the periodic seam, plus
    ordinary ones; returns (pos (3,n), owners)."""
    b = gen.bounds(p)
    nsub = p[0] * p[1] * p[2]
    owners = rng.integers(0, nsub, n)
    pos = np.zeros((3, n))
    for a in range(3):
        P = p[a]
        W = TWO_PI / P
        k = [(int(s) // [1, p[0], p[0] * p[1]][a]) % P for s in owners]
        k = np.array(k)
        lo, hi = b[a][k], b[a][k + 1]
        base = lo + (hi - lo) * rng.uniform(0, 1, n)
        kind = rng.integers(0, 12, n)
        x = base.copy()
        x[kind == 0] = lo[kind == 0]
        x[kind == 1] = np.nextafter(lo[kind == 1], -10)
        x[kind == 2] = hi[kind == 2]
        x[kind == 3] = np.nextafter(hi[kind == 3], -10)
        x[kind == 4] = lo[kind == 4] - 0.3 * W * rng.uniform(0, 1, (kind == 4).sum())
        x[kind == 5] = hi[kind == 5] + 0.3 * W * rng.uniform(0, 1, (kind == 5).sum())
        x[kind == 6] = np.where(k[kind == 6] == 0, -1e-300, x[kind == 6])
        x[kind == 7] = np.where(k[kind == 7] == P - 1, TWO_PI, x[kind == 7])
        pos[a] = x
    return pos, owners


@pytest.mark.parametrize("p,n", [((1, 1, 1), 5000), ((2, 2, 2), 30000), ((3, 2, 4), 50000),
                                 ((8, 8, 8), 120000), ((2, 1, 1), 3)])
def test_classify_scan_pack_and_compact_append_bit_exact(p, n):
    say(f"[test] migration bit-exact p={p} n={n}")
    from helpers import like, pool_from, send_for
    rng = np.random.default_rng(sum(p) * 1000 + n)
    pos, owners = special_positions(rng, p, n)
    nsub = p[0] * p[1] * p[2]
    vel = rng.standard_normal((3, n))
    tau = rng.uniform(0.01, 1.0, n)
    host = pool_from(pos, owners, nsub, vel=vel, tau=tau, extra=n // nsub + 64)
    ref_out = like(host, extra=n // 2 + 64)
    ref_send = send_for(nsub, cap_each=n // 4 + 64)
    odc = oracle.Decomp(p, gen.bounds(p))
    stay, f1 = oracle.partition(odc, host, ref_out, ref_send)
    f2 = oracle.append(odc, ref_send, stay, ref_out)

    dev = torch.device("cuda:0")
    pin = pm.DevicePool.from_host(host, dev)
    pout = pm.DevicePool.empty(ref_out.base, ref_out.cap, device=dev,
                               size=max(pin.size, ref_out.x.shape[1]))
    send = pm.DevicePool.empty(ref_send.base, ref_send.cap, device=dev)
    pin = pm.DevicePool.from_host(host, dev, size=pout.size)
    ctx = pm.Context(pout.size, send.size, nsub, device=dev)
    dc = pm.Decomp(p, gen.bounds(p))
    ctx.classify_scan_pack(dc, pin, send)
    ctx.compact_append(dc, pin, send, pout)
    flags = ctx.get_status()
    assert flags == (f1 | f2), (pm.flag_names(flags), f1 | f2)
    say(f"  flags {pm.flag_names(flags)}; migrants {int(ref_send.count.sum())}")
    compare_pools(send.to_host(), ref_send, nsub * 27, TWO_PI, 1.0, exact=True, what="send")
    compare_pools(pout.to_host(), ref_out, nsub, TWO_PI, 1.0, exact=True, what="out")


# ---------------------------------------------------------------------------
# fused step against the oracle
# ---------------------------------------------------------------------------

STEP_CASES = [
    ("C1", None, None, None, 1.0),
    ("C2", 40000, 32, None, 1.0),
    ("C2S", 60000, 32, (4, 4, 4), 1.0),
    ("C4", 300, 32, (4, 4, 4), 1.0),
    ("C3", 50000, 32, (4, 4, 4), 1.0),
]


@pytest.mark.parametrize("name,npart,n,p,dts", STEP_CASES)
def test_step_matches_oracle(name, npart, n, p, dts):
    say(f"[test] step vs oracle {name}")
    c = Case(name, npart, n, p, dt_scale=dts)
    if name == "C2S":
        c.params = pm.Params(min(c.dt, 0.015), c.g)
    pin = c.pin()
    send = c.send()
    pout = c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.step(c.field, c.dc, pin, pout, send, c.params)
    flags = ctx.get_status()
    ref_out, ref_send, stay, oflags = c.oracle_step(dt=c.params.dt)
    assert flags == oflags == 0, pm.flag_names(flags)
    delta = c.wl.L / c.wl.n
    compare_pools(send.to_host(), ref_send, c.dc.nsub * 27, c.wl.L, delta, what="send")
    ex, ev = compare_pools(pout.to_host(), ref_out, c.dc.nsub, c.wl.L, delta, what="out")
    say(f"  migrants {int(ref_send.count.sum())}; max err x {ex:.2e} v {ev:.2e}")
    # the input is left as it was
    h = pin.to_host()
    np.testing.assert_array_equal(h.x, c.host.x[:, :h.x.shape[1]])


def test_ten_steps_match_the_oracle():
    say("[test] ten steps C1")
    c = Case("C1")
    pa, send = c.pin(), c.send()
    pb = c.pout(pa.size)
    ctx = c.ctx(pa, send)
    host = c.host
    for k in range(10):
        ctx.step(c.field, c.dc, pa, pb, send, c.params)
        pa, pb = pb, pa
        ref_out, ref_send, _, of = c.oracle_step(pool=host)
        assert of == 0
        host = ref_out
    assert ctx.get_status() == 0
    compare_pools(pa.to_host(), host, c.dc.nsub, c.wl.L, c.wl.L / c.wl.n, tol=1e-11,
                  what="after 10 steps")


# ---------------------------------------------------------------------------
# internal identities: fused == plain, launch shapes, determinism, graphs
# ---------------------------------------------------------------------------

def run_plain(c, ctx, pin_host_copy, send, pout):
    ctx.interp_advance(c.field, pin_host_copy, c.params)
    ctx.classify_scan_pack(c.dc, pin_host_copy, send)
    ctx.compact_append(c.dc, pin_host_copy, send, pout)


@pytest.mark.parametrize("name,npart,n,p", [("C1", None, None, None),
                                            ("C2S", 80000, 32, (8, 8, 8)),
                                            ("C2", 50000, 32, (1, 1, 1))])
def test_fused_equals_plain_bitwise(name, npart, n, p):
    say(f"[test] fused == plain {name}")
    c = Case(name, npart, n, p)
    if name == "C2S":
        c.params = pm.Params(min(c.dt, 0.015), c.g)
    pin = c.pin()
    send_a, send_b = c.send(), c.send()
    out_a, out_b = c.pout(pin.size), c.pout(pin.size)
    ctx = c.ctx(pin, send_a)
    ctx.step(c.field, c.dc, pin, out_a, send_a, c.params)
    plain_in = c.pin()
    run_plain(c, ctx, plain_in, send_b, out_b)
    assert ctx.get_status() == 0
    assert_same_device_pools(out_a, out_b, c.dc.nsub, "out")
    assert_same_device_pools(send_a, send_b, c.dc.nsub * 27, "send")


@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_every_launch_shape_gives_identical_results(mode):
    say(f"[test] launch shapes, mode {mode}")
    c = Case("C2S", 70000, 32, (4, 2, 2), mode=mode)
    c.params = pm.Params(0.015, c.g)
    pin = c.pin()
    ref_out, ref_send = None, None
    ctx = c.ctx(pin, c.send())
    for wg, items in pm.SHAPES:
        # blocks per CU (0 = occupancy) and the tile order (0 = one ticket
        # counter; 3, 16 = XCD-cyclic blocks of that many tiles)
        for bpc, xb in ((0, 0), (1, 3), (0, 16)):
            say(f"  shape wg={wg} items={items} bpc={bpc} xcd_block={xb}")
            ctx.set_tuning(wg, items, bpc, xb)
            send, out = c.send(), c.pout(pin.size)
            ctx.step(c.field, c.dc, pin, out, send, c.params)
            assert ctx.get_status() == 0
            if ref_out is None:
                ref_out, ref_send = out, send
            else:
                assert_same_device_pools(out, ref_out, c.dc.nsub, f"out {wg}x{items}")
                assert_same_device_pools(send, ref_send, c.dc.nsub * 27, f"send {wg}x{items}")
            plain_in = c.pin()
            send2, out2 = c.send(), c.pout(pin.size)
            run_plain(c, ctx, plain_in, send2, out2)
            assert ctx.get_status() == 0
            assert_same_device_pools(out2, ref_out, c.dc.nsub, f"plain out {wg}x{items}")


def test_repeated_steps_are_deterministic():
    say("[test] determinism")
    c = Case("C2S", 100000, 32, (8, 4, 4))
    c.params = pm.Params(0.015, c.g)
    pin = c.pin()
    ctx = c.ctx(pin, c.send())
    ref = None
    for k in range(20):
        send, out = c.send(), c.pout(pin.size)
        ctx.step(c.field, c.dc, pin, out, send, c.params)
        if ref is None:
            ref = (out, send)
        else:
            assert_same_device_pools(out, ref[0], c.dc.nsub, f"out rep {k}")
            assert_same_device_pools(send, ref[1], c.dc.nsub * 27, f"send rep {k}")
    assert ctx.get_status() == 0


def test_graph_replays_match_eager():
    """Every replay (two graphs, one per ping-pong direction, three replays
    each, with eager torch work and synchronisations in between) against the
    eager step it stands for, bit for bit."""
    say("[test] graph replays")
    c = Case("C1")
    pa, send = c.pin(), c.send()
    pb = c.pout(pa.size)
    ctx = c.ctx(pa, send)
    ea, eb = c.pin(), c.pout(pa.size)
    ref = []
    for _ in range(6):
        ctx.step(c.field, c.dc, ea, eb, send, c.params)
        ea, eb = eb, ea
        ref.append(ea.to_host())
    ctx.set_graph(True)
    for k in range(6):
        ctx.step(c.field, c.dc, pa, pb, send, c.params)
        pa, pb = pb, pa
        torch.cuda.synchronize()
        _ = pa.x.sum().item()  # eager torch work between replays
        got = pa.to_host()
        np.testing.assert_array_equal(got.count, ref[k].count, err_msg=f"replay {k}")
        for q in range(c.dc.nsub):
            s = seg(ref[k], q)
            np.testing.assert_array_equal(got.x[:, s], ref[k].x[:, s], err_msg=f"replay {k}")
            np.testing.assert_array_equal(got.v[:, s], ref[k].v[:, s], err_msg=f"replay {k}")
            np.testing.assert_array_equal(got.id[s], ref[k].id[s], err_msg=f"replay {k}")
    ctx.set_graph(False)
    assert ctx.get_status() == 0


# ---------------------------------------------------------------------------
# error flags, forced from the host
# ---------------------------------------------------------------------------

def test_send_overflow_keeps_exact_counts_and_input_intact():
    say("[test] send overflow")
    c = Case("C2S", 40000, 32, (4, 4, 4))
    c.params = pm.Params(0.015, c.g)
    pin = c.pin()
    small = np.minimum(c.sc, 1)
    send = pm.DevicePool.empty(c.sb, small, device=c.dev, size=int((c.sb + c.sc).max()))
    out = c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.step(c.field, c.dc, pin, out, send, c.params)
    flags = ctx.get_status()
    assert flags & pm.SEND_OVERFLOW
    ref_out, ref_send, _, _ = c.oracle_step(dt=0.015)
    np.testing.assert_array_equal(send.to_host().count, ref_send.count)
    np.testing.assert_array_equal(out.to_host().count, ref_out.count)
    # regrow and retry from the intact input: identical to the oracle
    send2 = c.send()
    ctx.step(c.field, c.dc, pin, out, send2, c.params)
    assert ctx.get_status() == 0
    compare_pools(out.to_host(), ref_out, c.dc.nsub, c.wl.L, c.wl.L / c.wl.n)


def test_nonfinite_skip_and_halo_flags():
    say("[test] nonfinite / skip / halo")
    c = Case("C2", 5000, 32, (2, 2, 2))
    host = c.host
    host.x[0, int(host.base[0]) + 3] = np.nan
    pin = c.pin()
    send, out = c.send(), c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.step(c.field, c.dc, pin, out, send, c.params)
    assert ctx.get_status() & pm.NONFINITE
    assert int(out.count.sum()) == int(host.count.sum())
    # a huge step: particles jump beyond their neighbours, stencils leave the halo
    ctx.step(c.field, c.dc, pin, out, send, pm.Params(50.0, c.g))
    f = ctx.get_status()
    assert f & pm.SKIP and f & pm.HALO
    assert int(out.count.sum()) == int(host.count.sum())


def test_inconsistent_segment_table_is_a_no_op():
    say("[test] layout guard")
    c = Case("C1", 5000, 32)
    pin = c.pin()
    send, out = c.send(), c.pout(pin.size)
    ctx = c.ctx(pin, send)
    pin.count[0] = pin.cap[0] + 5  # count beyond capacity
    out.count.fill_(-7)
    ctx.step(c.field, c.dc, pin, out, send, c.params)
    assert ctx.get_status() & pm.LAYOUT
    assert int(out.count[0].item()) == -7
    pin.count[0] = int(c.host.count[0])
    ctx.step(c.field, c.dc, pin, out, send, c.params)
    assert ctx.get_status() == 0


def test_overlapping_segments_raise_layout():
    """Four segments over the same 4096 records, stepped with 1024-record
    tiles: 16 tiles, more than non-overlapping segments of that extent can
    give (4096/1024 + 4 + 2 look-back words are cleared), so the step must
    flag the layout and do nothing rather than read stale look-back words."""
    say("[test] overlapping segments")
    c = Case("C2S", 8000, 32, (2, 2, 1))
    n = 4096
    host = gen.empty_pool(np.zeros(4, dtype=np.int64), np.full(4, n, dtype=np.int64))
    host.x[:, :] = c.host.x[:, :n]
    host.v[:, :] = c.host.v[:, :n]
    host.tau[:] = c.host.tau[:n]
    host.id[:] = c.host.id[:n]
    host.count[:] = n
    pin = pm.DevicePool.from_host(host, c.dev)
    send = c.send()
    q = n // 4
    out = pm.DevicePool.empty(np.arange(4) * q, np.full(4, q), device=c.dev, size=n)
    ctx = pm.Context(n, send.size, 4, device=c.dev)
    ctx.set_tuning(256, 4)
    out.count.fill_(-7)
    ctx.step(c.field, c.dc, pin, out, send, c.params)
    assert ctx.get_status() & pm.LAYOUT
    assert int(out.count[0].item()) == -7


# ---------------------------------------------------------------------------
# mixed precision against the float64 oracle
# ---------------------------------------------------------------------------

def test_mixed_precision_error_against_the_fp64_oracle():
    say("[test] mixed precision")
    c = Case("C5", 40000, 64, (4, 4, 4), mode="mixed")
    pin = c.pin()
    send, out = c.send(), c.pout(pin.size)
    ctx = c.ctx(pin, send)
    ctx.step(c.field, c.dc, pin, out, send, c.params)
    assert ctx.get_status() == 0
    ref_out, _, _, _ = c.oracle_step()
    got = out.to_host()
    np.testing.assert_array_equal(np.sort(got.id[:int(got.count.sum())] if c.dc.nsub == 1
                                          else np.concatenate([got.id[seg(got, q)]
                                                               for q in range(c.dc.nsub)])),
                                  np.arange(int(c.host.count.sum()), dtype=np.uint64))
    # compare per id (ownership may differ for particles within ~1e-6 cell of a face)
    gid = np.concatenate([got.id[seg(got, q)] for q in range(c.dc.nsub)])
    gx = np.concatenate([got.x[:, seg(got, q)] for q in range(c.dc.nsub)], axis=1)
    gv = np.concatenate([got.v[:, seg(got, q)] for q in range(c.dc.nsub)], axis=1)
    rid = np.concatenate([ref_out.id[seg(ref_out, q)] for q in range(c.dc.nsub)])
    rx = np.concatenate([ref_out.x[:, seg(ref_out, q)] for q in range(c.dc.nsub)], axis=1)
    rv = np.concatenate([ref_out.v[:, seg(ref_out, q)] for q in range(c.dc.nsub)], axis=1)
    gi, ri = np.argsort(gid), np.argsort(rid)
    delta = c.wl.L / c.wl.n
    dx = np.abs(np.mod(gx[:, gi] - rx[:, ri] + np.pi, 2 * np.pi) - np.pi).max() / delta
    dv = np.abs(gv[:, gi].astype(np.float64) - rv[:, ri]).max()
    say(f"  mixed vs fp64: |dx|/cell {dx:.2e}, |dv|/u_rms {dv:.2e}")
    assert dv <= 1e-6 and dx <= 1e-6
