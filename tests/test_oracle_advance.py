"""Pins of the oracle's particle advance (Sect. 2.2: dX/dt = V,
dV/dt = -(1/tau)(V - U(X)) + g, two-stage second-order Runge-Kutta) against
closed forms, a fixed point, and convergence order on a nonlinear field
solved independently by scipy."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle

N = 64
L = 64.0


def const_field(u, n=N, halo=0):
    st = n + 2 * halo
    return oracle.Field([np.full(st ** 3, float(c)) for c in u], n, halo, L)


def run(field, x, v, tau, dt, g, steps):
    for _ in range(steps):
        x, v, flags = oracle.advance(field, x, v, tau, dt, g)
        assert flags == 0
    return x, v


def test_uniform_flow_translates_exactly():
    u = (0.25, -0.5, 0.125)
    f = const_field(u)
    rng = np.random.default_rng(10)
    x0 = np.round(rng.uniform(8, 56, (3, 300)) * 1024) / 1024
    v0 = np.tile(np.array(u)[:, None], (1, 300))
    dt = 1.0 / 64
    x, v = x0, v0
    for n in range(1, 11):
        x, v = run(f, x, v, np.full(300, 0.5), dt, (0, 0, 0), 1)
        np.testing.assert_array_equal(x, x0 + n * dt * np.array(u)[:, None])
        np.testing.assert_array_equal(v, v0)


@pytest.mark.parametrize("tau,dt", [(0.2, 0.01), (0.05, 0.01), (1.0, 0.003)])
def test_drag_in_constant_flow_matches_discrete_closed_form(tau, dt):
    # one step maps V - u to rho (V - u) with rho = 1 - h + h^2/2, h = dt/tau,
    # and moves X by dt u + dt (1 - h/2)(V - u)
    u = np.array([0.3, -0.7, 1.1])
    f = const_field(u)
    rng = np.random.default_rng(11)
    npart = 64
    x0 = rng.uniform(5, 60, (3, npart))
    v0 = rng.standard_normal((3, npart))
    h = dt / tau
    rho = 1 - h + h * h / 2
    x, v = x0, v0
    for n in (1, 5, 20, 50):
        x, v = run(f, x0, v0, np.full(npart, tau), dt, (0, 0, 0), n)
        vn = u[:, None] + rho ** n * (v0 - u[:, None])
        xn = x0 + n * dt * u[:, None] + dt * (1 - h / 2) * (v0 - u[:, None]) * (1 - rho ** n) / (1 - rho)
        assert np.max(np.abs(v - vn)) <= 1e-13 * max(1.0, np.max(np.abs(vn)))
        assert np.max(np.abs(x - xn)) <= 1e-13 * np.max(np.abs(xn))


def test_second_order_convergence_to_the_continuous_solution():
    # v(t) = u + (v0 - u) exp(-t/tau); x(t) = x0 + u t + tau (v0 - u)(1 - exp(-t/tau))
    u = np.array([0.4, 0.0, -0.2])
    f = const_field(u)
    tau, T = 0.1, 0.4
    x0 = np.array([[20.0], [30.0], [40.0]])
    v0 = np.array([[1.0], [-1.0], [0.5]])
    ve = u[:, None] + (v0 - u[:, None]) * math.exp(-T / tau)
    xe = x0 + u[:, None] * T + tau * (v0 - u[:, None]) * (1 - math.exp(-T / tau))
    errs = []
    for nsteps in (40, 80, 160):
        x, v = run(f, x0, v0, np.array([tau]), T / nsteps, (0, 0, 0), nsteps)
        errs.append(np.max(np.abs(v - ve)) + np.max(np.abs(x - xe)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


def test_terminal_velocity_under_gravity_is_a_fixed_point():
    u = (0.5, -0.25, 0.125)
    g = (0.0, 0.0, -1.0)
    tau = 0.25
    f = const_field(u)
    vt = np.array(u) + tau * np.array(g)
    x0 = np.array([[10.0, 20.5], [11.25, 30.0], [12.0, 40.75]])
    v0 = np.tile(vt[:, None], (1, 2))
    dt = 1.0 / 32
    x, v = run(f, x0, v0, np.full(2, tau), dt, g, 8)
    np.testing.assert_array_equal(v, v0)
    np.testing.assert_array_equal(x, x0 + 8 * dt * vt[:, None])


def test_gravity_changes_velocity_by_g_dt_from_rest_in_still_fluid_limit():
    # tau -> large: drag vanishes and one Heun step gives V' = V + g dt exactly
    f = const_field((0.0, 0.0, 0.0))
    g = (0.0, 0.0, -1.0)
    x0 = np.array([[10.0], [10.0], [10.0]])
    v0 = np.zeros((3, 1))
    x, v = run(f, x0, v0, np.array([1e300]), 0.5, g, 1)
    np.testing.assert_array_equal(v[:, 0], [0.0, 0.0, -0.5])
    np.testing.assert_array_equal(x[:, 0], [10.0, 10.0, 10.0 - 0.125])


COEFS = [(0.2, 0.0, 0.01, -0.02, 0.0, 0.003, 0.0, 0.0002),
         (-0.1, 0.015, 0.0, 0.01, -0.002, 0.0, 0.001, 0.0),
         (0.05, -0.01, 0.02, 0.0, 0.0, 0.0, -0.0015, 0.0001)]


def analytic(coef, x, y, z):
    a, b, c, d, e, f, g, h = coef
    return a + b * x + c * y + d * z + e * x * y + f * y * z + g * x * z + h * x * y * z


def test_second_order_on_a_nonlinear_field_against_scipy():
    # halo-mode field that is trilinear over the whole box: the interpolant equals
    # the analytic field everywhere, so the discrete ODE is the continuous one
    idx = np.arange(-1, N + 1) + 0.5
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    f = oracle.Field([analytic(c, x, y, z).reshape(-1) for c in COEFS], N, 1, L)
    tau, T = 0.3, 2.0
    g = (0.0, 0.0, -0.5)
    x0 = np.array([30.0, 31.0, 32.0])
    v0 = np.array([0.1, -0.2, 0.05])

    def rhs(t, s):
        X, V = s[:3], s[3:]
        U = np.array([analytic(c, *X) for c in COEFS])
        return np.concatenate([V, (U - V) / tau + np.array(g)])

    ref = solve_ivp(rhs, (0, T), np.concatenate([x0, v0]), method="DOP853",
                    rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for nsteps in (50, 100, 200):
        x1, v1 = run(f, x0[:, None].copy(), v0[:, None].copy(), np.array([tau]),
                     T / nsteps, g, nsteps)
        errs.append(np.max(np.abs(np.concatenate([x1[:, 0], v1[:, 0]]) - ref)))
    assert errs[2] < 1e-4
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs
