"""Pins of the oracle's MAC-staggered interpolation: component c is stored on
the faces normal to axis c (offset 0 along axis c, 1/2 of a cell along the
others), as a marker-and-cell fluid solver (Sect. 2.1) leaves it.

Setup as for the collocated pins: L = N = 64 (cell width 1) and dyadic
positions.  A field trilinear in space, sampled at each component's own node
positions, must come back bit for bit; the same samples read as collocated
must not (the half-cell shift is visible), and a node of each component
returns its stored value.
"""
import numpy as np

import oracle

N = 64
L = 64.0
COEFS = [(3, 2, -1, 1, 1, 0, -2, 1), (-5, 1, 4, -3, 0, 2, 1, -1), (7, -2, 0, 5, -1, 1, 0, 2)]


def analytic(coef, x, y, z):
    a, b, c, d, e, f, g, h = coef
    return a + b * x + c * y + d * z + e * x * y + f * y * z + g * x * z + h * x * y * z


def mac_field(halo):
    lo, hi = (-1, N + 1) if halo else (0, N)
    idx = np.arange(lo, hi, dtype=np.float64)
    comps = []
    for c in range(3):
        pos = [idx + (0.0 if a == c else 0.5) for a in range(3)]
        z, y, x = np.meshgrid(pos[2], pos[1], pos[0], indexing="ij")
        comps.append(analytic(COEFS[c], x, y, z).reshape(-1))
    return comps


def dyadic_points(rng, n, lo, hi, denom=64):
    return np.round(rng.uniform(lo, hi, (3, n)) * denom) / denom


def test_trilinear_mac_field_is_reproduced_exactly():
    f = oracle.Field(mac_field(halo=1), N, 1, L, stagger=True)
    X = dyadic_points(np.random.default_rng(11), 4000, 0.0, L - 1.0 / 64)
    U, flags = oracle.interp(f, X)
    assert flags == 0
    for c in range(3):
        np.testing.assert_array_equal(U[c], analytic(COEFS[c], *X))


def test_periodic_mac_field_away_from_the_seam():
    f = oracle.Field(mac_field(halo=0), N, 0, L, stagger=True)
    X = dyadic_points(np.random.default_rng(12), 4000, 1.0, L - 1.0 - 1.0 / 64)
    U, flags = oracle.interp(f, X)
    assert flags == 0
    for c in range(3):
        np.testing.assert_array_equal(U[c], analytic(COEFS[c], *X))


def test_collocated_reading_of_the_same_samples_differs():
    u = mac_field(halo=1)
    X = dyadic_points(np.random.default_rng(13), 500, 1.0, L - 2.0)
    Um, _ = oracle.interp(oracle.Field(u, N, 1, L, stagger=True), X)
    Uc, _ = oracle.interp(oracle.Field(u, N, 1, L), X)
    for c in range(3):
        assert np.abs(Um[c] - Uc[c]).max() > 0.1


def test_face_nodes_return_their_values():
    rng = np.random.default_rng(14)
    u = [rng.standard_normal(N ** 3) for _ in range(3)]
    f = oracle.Field(u, N, 0, L, stagger=True)
    ijk = rng.integers(1, N - 1, (3, 200))
    for c in range(3):
        X = ijk.astype(np.float64) + np.array([0.0 if a == c else 0.5 for a in range(3)])[:, None]
        U, _ = oracle.interp(f, X)
        node = ijk[0] + N * (ijk[1] + N * ijk[2])
        np.testing.assert_array_equal(U[c], u[c][node])
