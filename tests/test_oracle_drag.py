"""Pins of the oracle's nonlinear drag law (Sect. 2.2): dV/dt = -(f/tau)(V - U) + g,
f = 1 + 0.15 Re_p^0.687, Re_p = 2 r |V - U| / nu, tau = (2/9)(rho_p/rho) r^2 / nu.

* Stokes limit: with nu so large that Re_p^0.687 underflows against 1, the
  step equals the Stokes step bit for bit.
* Terminal velocity: in a uniform flow under gravity, the slip w that solves
  w f(w) = tau |g| (found by bracketing, independently of the oracle) is a
  fixed point of the step: V stays, X moves by dt V.
* Order 2 against the exact ODE: in still fluid, one Heun step from V0 differs
  from a tight solve_ivp solution by O(dt^3) (halving dt divides the error by
  about 8), while the Stokes step differs by O(dt) from that solution.  A wrong
  constant, exponent, radius or slip would leave an O(dt) error.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

import oracle

NU = 1.5e-5
RHO = 843.0


def uniform_field(u, n=4, L=2 * math.pi):
    return oracle.Field([np.full(n ** 3, float(c)) for c in u], n, 0, L)


def slip_speed_re(w, tau):
    # Re_p of a particle of relaxation time tau at slip speed w
    r = math.sqrt(tau * NU * 9.0 / 2.0 / RHO)
    return w * 2.0 * r / NU


def test_stokes_limit_is_bitwise_stokes():
    rng = np.random.default_rng(7)
    n = 8
    f = oracle.Field([rng.standard_normal(n ** 3) for _ in range(3)], n, 0)
    x = rng.uniform(0, 2 * math.pi, (3, 200))
    v = rng.standard_normal((3, 200))
    tau = np.exp(rng.uniform(math.log(0.01), 0.0, 200))
    xs, vs, _ = oracle.advance(f, x, v, tau, 0.01, (0.0, 0.0, -1.0))
    xn, vn, _ = oracle.advance(f, x, v, tau, 0.01, (0.0, 0.0, -1.0), drag="nonlinear",
                               nu=1e300)
    assert np.array_equal(xs, xn) and np.array_equal(vs, vn)
    # and the law matters at the paper's parameters
    _, vp, _ = oracle.advance(f, x, v, tau, 0.01, (0.0, 0.0, -1.0), drag="nonlinear")
    assert np.abs(vp - vs).max() > 1e-4


@pytest.mark.parametrize("tau", [0.01, 0.1, 1.0])
def test_terminal_velocity_is_a_fixed_point(tau):
    U0 = np.array([0.3, -0.2, 0.1])
    g = np.array([0.0, 0.0, -9.81])
    gn = float(np.linalg.norm(g))
    w = brentq(lambda w: w * (1 + 0.15 * slip_speed_re(w, tau) ** 0.687) - tau * gn,
               0.0, tau * gn, xtol=1e-15, rtol=1e-15)
    assert w < tau * gn * 0.999          # the correction is not negligible here
    V = U0 + g / gn * w
    x = np.array([[1.0], [2.0], [3.0]])
    f = uniform_field(U0)
    x1, v1, flags = oracle.advance(f, x, V[:, None], [tau], 1e-3, g, drag="nonlinear")
    assert flags == 0
    assert np.allclose(v1[:, 0], V, rtol=0, atol=1e-13 * max(1.0, w))
    assert np.allclose(x1[:, 0], x[:, 0] + 1e-3 * V, rtol=0, atol=1e-15)


@pytest.mark.parametrize("tau,w0", [(0.05, 2.0), (1.0, 0.7)])
def test_heun_is_second_order_for_the_nonlinear_law(tau, w0):
    f0 = uniform_field((0.0, 0.0, 0.0))

    def rhs(t, y):
        w = abs(y[0])
        return [-(1 + 0.15 * slip_speed_re(w, tau) ** 0.687) * y[0] / tau]

    errs, errs_stokes = [], []
    for dt in (0.02 * tau, 0.01 * tau, 0.005 * tau):
        exact = solve_ivp(rhs, (0, dt), [w0], rtol=1e-13, atol=1e-15, method="DOP853").y[0, -1]
        x = np.array([[1.0], [1.0], [1.0]])
        v = np.array([[w0], [0.0], [0.0]])
        _, vn, _ = oracle.advance(f0, x, v, [tau], dt, drag="nonlinear")
        _, vs, _ = oracle.advance(f0, x, v, [tau], dt)
        errs.append(abs(vn[0, 0] - exact))
        errs_stokes.append(abs(vs[0, 0] - exact))
    for a, b in zip(errs, errs[1:]):
        assert 6.0 < a / b < 10.0
    for a, b in zip(errs_stokes, errs_stokes[1:]):
        assert 1.8 < a / b < 2.2
    assert errs[-1] < 1e-3 * errs_stokes[-1]
