"""The synthetic input generator: spectrum shape (estimator of Sect. 3.1.1),
zero divergence, unit rms, determinism, and pool layout."""
import math

import numpy as np
import pytest

from paper_2604_11008_amd import gen


@pytest.fixture(scope="module")
def field64():
    return gen.spectral_field(64, 4, 8, gen.seeds(0)[0])


def test_unit_rms(field64):
    ms = sum(float(np.mean(u * u)) for u in field64) / 3
    assert abs(ms - 1.0) < 1e-12


def test_deterministic(field64):
    again = gen.spectral_field(64, 4, 8, gen.seeds(0)[0])
    for a, b in zip(field64, again):
        np.testing.assert_array_equal(a, b)


def test_divergence_free_in_spectral_space(field64):
    n = 64
    f = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(f, f, f, indexing="ij")
    uh = [np.fft.fftn(u) for u in field64]
    div = kx * uh[0] + ky * uh[1] + kz * uh[2]
    mag = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2) * np.sqrt(sum(np.abs(c) ** 2 for c in uh))
    assert np.max(np.abs(div)) <= 1e-10 * np.max(mag)


def test_spectrum_follows_the_model_shape(field64):
    e = gen.shell_spectrum(field64, kmax_out=12)
    model = gen.model_spectrum(np.arange(13), 4)
    # shells 3..7 are complete (shell 8 is cut at |k| = 8)
    ratio = e[3:8] / model[3:8]
    assert np.max(np.abs(ratio / np.median(ratio) - 1)) < 0.15
    assert np.all(e[9:] < 1e-20 * e.max())
    # Parseval: half the mean square speed equals the summed shell energy up to
    # the shell-weighting of the estimator
    ke = 0.5 * sum(float(np.mean(u * u)) for u in field64)
    assert 0.7 < e.sum() / ke < 1.4


def test_pool_layout_and_canonical_order():
    wl = gen.make_workload("C1", np_override=5000, n_override=32)
    pool = wl.pool
    assert np.all(np.diff(pool.base) >= 0)
    assert np.all(pool.base[:-1] + pool.cap[:-1] <= pool.base[1:])
    assert np.all(pool.count <= pool.cap)
    ids = np.concatenate([pool.id[pool.segment(s)] for s in range(8)])
    np.testing.assert_array_equal(np.sort(ids), np.arange(5000, dtype=np.uint64))
    for s in range(8):
        x = pool.x[:, pool.segment(s)]
        assert np.all((x >= 0) & (x < wl.L))
        np.testing.assert_array_equal(gen.owner(x, wl.bounds, wl.p), s)
        cell = np.floor(x * (wl.n / wl.L)).astype(np.int64)
        key = gen.cell_key(cell[0], cell[1], cell[2])
        assert np.all(np.diff(key) >= 0)


def test_cell_key_orders_x_pairs_then_z_order():
    i, j, k = np.meshgrid(np.arange(4), np.arange(2), np.arange(2), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    order = np.argsort(gen.cell_key(i, j, k), kind="stable")
    cells = list(zip(i[order], j[order], k[order]))
    # x pairs are the leaves; the pairs themselves follow the Z-order of
    # (i/2, j, k): x pair 0, x pair 1, then j, then k
    assert cells[:4] == [(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)]
    assert cells[4:8] == [(0, 1, 0), (1, 1, 0), (2, 1, 0), (3, 1, 0)]
    assert cells[8:10] == [(0, 0, 1), (1, 0, 1)]
    assert len(set(gen.cell_key(i, j, k))) == i.size


def test_blob_and_lognormal_distributions():
    g = gen.rng(gen.seeds(2)[1])
    pos = gen.blob_positions(g, 100000, 64)
    assert pos.shape == (3, 100000) and np.all((pos >= 0) & (pos < 2 * math.pi))
    b = gen.bounds((4, 4, 4))
    pos = gen.lognormal_positions(gen.rng(gen.seeds(3)[1]), (4, 4, 4), b, median=200)
    s = gen.owner(pos, b, (4, 4, 4))
    counts = np.bincount(s, minlength=64)
    assert 100 < np.median(counts) < 400


def test_tau_distributions():
    g = gen.rng(1)
    t = gen.draw_tau(g, 100000, ("loguniform", 0.01, 1.0))
    assert t.min() >= 0.01 and t.max() <= 1.0
    assert abs(np.median(np.log(t)) - math.log(0.1)) < 0.05


@pytest.mark.parametrize("name,kw", [
    ("C2S", dict(np_override=60000, n_override=64)),
    ("C4", dict(np_override=500, n_override=64)),
    ("C5", dict(np_override=1 << 17, n_override=64))])
@pytest.mark.parametrize("order", ["canonical", "morton", "rowmajor", "shuffled"])
def test_torch_ordering_builds_the_same_pool(name, kw, order):
    """The torch path of build_pool (run on the CPU here; on the GPU for the
    large workloads) gives the numpy lexsort's pool record for record."""
    a = gen.make_workload(name, order=order, **kw)
    b = gen.make_workload(name, order=order, sort_device="cpu", **kw)
    for f in ("x", "tau", "id", "base", "cap", "count"):
        np.testing.assert_array_equal(getattr(a.pool, f), getattr(b.pool, f), err_msg=f)


def test_node_values_are_the_mode_sum_at_cell_centres():
    """Each stored value is the real field sum over the generated modes,
    2 Re(u_hat e^{i k.x}) per mode, evaluated at the cell centre (j + 1/2) h,
    scaled to unit rms; by Parseval (all modes below Nyquist) the grid's mean
    square before scaling is the sum of 2 |u_hat|^2."""
    n, k0, kmax = 32, 2, 4
    seed = gen.seeds(3)[0]
    u = gen.spectral_field(n, k0, kmax, seed)
    kv, uh = gen.spectral_modes(k0, kmax, seed)
    scale = 1.0 / math.sqrt(sum(float((2 * np.abs(uh[:, c]) ** 2).sum()) for c in range(3)) / 3)
    rng = np.random.default_rng(11)
    ijk = rng.integers(0, n, (3, 200))
    centres = (ijk + 0.5) * (2 * math.pi / n)
    ph = np.exp(1j * (kv.astype(np.float64) @ centres))
    for c in range(3):
        exact = scale * 2 * np.real(uh[:, c] @ ph)
        np.testing.assert_allclose(u[c][ijk[2], ijk[1], ijk[0]], exact, rtol=0, atol=1e-12)
