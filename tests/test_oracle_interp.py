"""Pins of the oracle's trilinear interpolation (Sect. 2.2: U(X) from the
eight surrounding cell-centre values) against closed forms and special cases.

Setup for exact checks: L = N = 64, so the cell width is 1, nodes sit at
i + 1/2 and every dyadic position gives exact weights.  A field that is
trilinear in space (a + bx + cy + dz + exy + fyz + gxz + hxyz) is reproduced
exactly by trilinear interpolation, so with small integer coefficients and
dyadic positions the oracle must return the analytic value bit for bit.
"""
import numpy as np
import pytest

import oracle

N = 64
L = 64.0


def analytic(coef, x, y, z):
    a, b, c, d, e, f, g, h = coef
    return a + b * x + c * y + d * z + e * x * y + f * y * z + g * x * z + h * x * y * z


def node_field(coefs, n=N, halo=0, width=1.0):
    """Analytic fields sampled at cell centres; halo adds nodes -1 and n."""
    lo, hi = (-1, n + 1) if halo else (0, n)
    idx = (np.arange(lo, hi) + 0.5) * width
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    return [analytic(c, x, y, z).reshape(-1) for c in coefs]


COEFS = [(3, 2, -1, 1, 1, 0, -2, 1), (-5, 1, 4, -3, 0, 2, 1, -1), (7, -2, 0, 5, -1, 1, 0, 2)]


def dyadic_points(rng, n, lo, hi, denom=64):
    return np.round(rng.uniform(lo, hi, (3, n)) * denom) / denom


def test_trilinear_field_is_reproduced_exactly_in_halo_mode():
    f = oracle.Field(node_field(COEFS, halo=1), N, 1, L)
    X = dyadic_points(np.random.default_rng(1), 4000, 0.0, L - 1.0 / 64)
    U, flags = oracle.interp(f, X)
    assert flags == 0
    for c in range(3):
        np.testing.assert_array_equal(U[c], analytic(COEFS[c], *X))


def test_trilinear_field_is_reproduced_exactly_away_from_the_seam():
    f = oracle.Field(node_field(COEFS, halo=0), N, 0, L)
    X = dyadic_points(np.random.default_rng(2), 4000, 0.5, L - 0.5 - 1.0 / 64)
    U, flags = oracle.interp(f, X)
    assert flags == 0
    for c in range(3):
        np.testing.assert_array_equal(U[c], analytic(COEFS[c], *X))


def test_node_values_are_returned_unchanged():
    rng = np.random.default_rng(3)
    u = [rng.standard_normal(N ** 3) for _ in range(3)]
    f = oracle.Field(u, N, 0, L)
    ijk = rng.integers(0, N, (3, 500))
    X = ijk + 0.5
    U, _ = oracle.interp(f, X)
    flat = ijk[0] + N * (ijk[1] + N * ijk[2])
    for c in range(3):
        np.testing.assert_array_equal(U[c], u[c][flat])


def test_constant_field_is_exact_anywhere():
    u = [np.full(N ** 3, 0.375), np.full(N ** 3, -1.25), np.full(N ** 3, 2.0)]
    f = oracle.Field(u, N, 0, L)
    X = dyadic_points(np.random.default_rng(4), 2000, 0.0, L - 1.0 / 64)
    U, _ = oracle.interp(f, X)
    np.testing.assert_array_equal(U[0], 0.375)
    np.testing.assert_array_equal(U[1], -1.25)
    np.testing.assert_array_equal(U[2], 2.0)


def test_periodic_seam_mixes_last_and_first_node():
    # x-component equal to the node's i index, constant in y and z
    i = np.arange(N, dtype=np.float64)
    u0 = np.broadcast_to(i[None, None, :], (N, N, N)).reshape(-1).copy()
    zero = np.zeros(N ** 3)
    f = oracle.Field([u0, zero, zero], N, 0, L)
    # x = L - 1/4: a quarter of the way from node 63 (at 63.5) to node 0 (at 64.5)
    # x = 1/4: three quarters of the way from node 63 (at -0.5) to node 0
    X = np.array([[L - 0.25, 0.25], [10.5, 10.5], [3.5, 3.5]])
    U, flags = oracle.interp(f, X)
    assert flags == 0
    np.testing.assert_array_equal(U[0], [47.25, 15.75])


def test_axes_are_not_transposed():
    # a field varying along one axis only must interpolate along that axis only
    for axis in range(3):
        coef = [0] * 8
        coef[1 + axis] = 1  # u = x, y or z
        f = oracle.Field(node_field([coef, coef, coef], halo=1), N, 1, L)
        X = np.array([[10.25], [20.75], [30.125]])
        U, _ = oracle.interp(f, X)
        assert U[0, 0] == X[axis, 0]


def test_halo_flag_outside_stored_nodes():
    f = oracle.Field(node_field(COEFS, halo=1), N, 1, L)
    inside = np.array([[-0.5, L + 0.49], [1.0, 1.0], [1.0, 1.0]])
    _, flags = oracle.interp(f, inside)
    assert flags == 0
    for bad in (-0.51, L + 0.5, -np.inf):
        _, flags = oracle.interp(f, np.array([[bad], [1.0], [1.0]]))
        assert flags == oracle.HALO, bad


def test_periodic_addressable_range_and_nan():
    u = [np.ones(N ** 3)] * 3
    f = oracle.Field(u, N, 0, L)
    _, flags = oracle.interp(f, np.array([[-L + 0.5, 2 * L - 0.6], [1.0, 1.0], [1.0, 1.0]]))
    assert flags == 0
    _, flags = oracle.interp(f, np.array([[-L - 1.0], [1.0], [1.0]]))
    assert flags == oracle.HALO
    U, flags = oracle.interp(f, np.array([[np.nan], [1.0], [1.0]]))
    assert flags == 0 and np.isnan(U).all()


@pytest.mark.parametrize("halo", [0, 1])
def test_interpolant_is_continuous_across_cell_faces(halo):
    rng = np.random.default_rng(5)
    n = 16
    st = n + 2 * halo
    u = [rng.standard_normal(st ** 3) for _ in range(3)]
    f = oracle.Field(u, n, halo, 2 * np.pi)
    dx = 2 * np.pi / n
    faces = (np.arange(1, n - 1) + 0.5) * dx  # node planes are the interpolant's cell faces
    X = np.stack([faces, np.full_like(faces, 1.3), np.full_like(faces, 2.1)])
    eps = 1e-9
    Ua, _ = oracle.interp(f, X - np.array([[eps], [0], [0]]))
    Ub, _ = oracle.interp(f, X + np.array([[eps], [0], [0]]))
    assert np.max(np.abs(Ua - Ub)) < 1e-6


def test_spectral_field_is_approximated_to_second_order():
    """On the generator's spectral field (cell-centre samples of a finite mode
    sum) the interpolant approaches the continuous field: at every point the
    error stays within the tensor-product bound of linear interpolation,
    sum over axes of t_a (1 - t_a) h^2 / 2 max |d^2 u / dx_a^2| (t_a the
    fraction of the cell below the point, the second derivative bounded by
    the amplitudes times k_a^2), and halving the cell divides the rms error by
    four.  A node convention off by any fraction of a cell leaves an error of
    first order."""
    from paper_2604_11008_amd import gen
    k0, kmax = 2, 4
    seed = gen.seeds(0)[0]
    kv, uh = gen.spectral_modes(k0, kmax, seed)
    kf = kv.astype(np.float64)
    scale = 1.0 / np.sqrt(sum(float((2 * np.abs(uh[:, c]) ** 2).sum()) for c in range(3)) / 3)
    L2 = 2 * np.pi
    X = np.random.default_rng(7).uniform(0.0, L2, (3, 4000))
    ph = np.exp(1j * (kf @ X))
    exact = [scale * 2 * np.real(uh[:, c] @ ph) for c in range(3)]
    d2max = [[scale * float((2 * np.abs(uh[:, c]) * kf[:, a] ** 2).sum()) for a in range(3)]
             for c in range(3)]
    rms = []
    for n in (32, 64, 128):
        h = L2 / n
        f = oracle.Field([a.reshape(-1) for a in gen.spectral_field(n, k0, kmax, seed)], n, 0, L2)
        U, flags = oracle.interp(f, X)
        assert flags == 0
        t = np.mod(X / h - 0.5, 1.0)
        err = []
        for c in range(3):
            e = np.abs(U[c] - exact[c])
            bound = sum(t[a] * (1 - t[a]) * h * h / 2 * d2max[c][a] for a in range(3))
            assert np.all(e <= bound + 1e-13), (n, c, float(np.max(e / bound)))
            err.append(np.sqrt(np.mean(e * e)))
        rms.append(max(err))
    for coarse, fine in zip(rms, rms[1:]):
        assert 3.6 < coarse / fine < 4.4, rms
