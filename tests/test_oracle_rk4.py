"""Pins for the oracle's classic RK4 integrator and the RK4 sampler built on it (the sampler ODE
of eq. 8; RK4 with 12 steps is what the paper times in "Convergence and Performance").

Each pin is fixed by mathematics, not by the code under test:
  * linear ODE x' = a x: one RK4 step multiplies by the degree-4 Taylor polynomial of e^{ah};
  * time-only field x' = g(t): RK4 reduces to Simpson's rule, exact for cubics and off by
    h^4 / 120 for g = t^4 (the Simpson error term);
  * x' = x^2 from 1/2 reaches exactly 1 at t = 1, and the error falls 16x per halving of h;
  * the network sampler agrees with scipy's DOP853 solve of the same ODE to its error bound.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2512_13965_amd import inputs


@pytest.mark.parametrize("K", [1, 3, 12])
def test_linear_ode_is_taylor_polynomial(orc, K):
    a = np.array([-3.0, -0.5, 0.7, 2.0, 5.0])
    x0 = np.array([1.0, -2.0, 0.5, 3.0, -1.5])
    z = a / K
    growth = 1.0 + z + z**2 / 2.0 + z**3 / 6.0 + z**4 / 24.0
    x = orc.rk4_solve(lambda x, t: a * x, x0, K)
    np.testing.assert_allclose(x, x0 * growth**K, rtol=1e-13)


@pytest.mark.parametrize("K", [1, 2, 12])
def test_time_only_field_is_simpson(orc, K):
    h = 1.0 / K
    # a cubic in t is integrated exactly: int_0^1 (1 - 2t + 3t^2 - 4t^3) dt = 1 - 1 + 1 - 1 = 0
    g3 = lambda x, t: np.full_like(x, 1.0 - 2.0 * t + 3.0 * t * t - 4.0 * t**3)
    x = orc.rk4_solve(g3, np.array([0.25]), K)
    assert abs(x[0] - 0.25) < 1e-14
    # t^4: Simpson's composite error is (b - a) h^4 f''''/2880 = h^4 / 120 (overestimate)
    x = orc.rk4_solve(lambda x, t: np.full_like(x, t**4), np.array([0.0]), K)
    assert abs(x[0] - (0.2 + h**4 / 120.0)) < 1e-14


def test_nonlinear_autonomous_order_four(orc):
    # x' = x^2, x(0) = 1/2  ->  x(t) = 1 / (2 - t), x(1) = 1
    errs = [abs(orc.rk4_solve(lambda x, t: x * x, np.array([0.5]), K)[0] - 1.0) for K in (4, 8, 16, 32)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(13.0 < r < 18.0 for r in ratios), ratios


def test_nonautonomous_coupled_order_four(orc):
    # x' = -t y, y' = t x: rotation by angle t^2 / 2, |x|^2 conserved by the flow
    f = lambda s, t: np.array([-t * s[1], t * s[0]])
    exact = np.array([math.cos(0.5), math.sin(0.5)])
    errs = [np.abs(orc.rk4_solve(f, np.array([1.0, 0.0]), K) - exact).max() for K in (4, 8, 16)]
    assert 13.0 < errs[0] / errs[1] < 19.0 and 13.0 < errs[1] / errs[2] < 19.0


def test_zero_network_gives_z_plus_bias(orc):
    w = inputs.random_weights(32, seed=3)
    for l in range(5):
        w.W[l][:] = 0.0
    cond = inputs.transmission_conditions(20, seed=6)
    z = inputs.noise(20, seed=7).astype(np.float64)
    for K in (1, 12):
        x = orc.sample_raw_rk4(w, cond, K, z)
        np.testing.assert_allclose(x, z.T + w.b[4][None, :].astype(np.float64), atol=1e-13)


@pytest.fixture(scope="module")
def ode_case():
    n = 6
    w = inputs.random_weights(32, seed=21)
    cond = inputs.transmission_conditions(n, seed=22)
    z = inputs.noise(n, seed=23).astype(np.float64)
    return w, cond, z


def _dop853(orc, w, cond, z):
    condf = orc.condition_features(cond)
    n = z.shape[1]

    def rhs(t, y):
        return orc.velocity(w, y.reshape(n, 5), t, condf).reshape(-1)

    sol = solve_ivp(rhs, (0.0, 1.0), z.T.reshape(-1), method="DOP853", rtol=1e-13, atol=1e-13)
    assert sol.success
    return sol.y[:, -1].reshape(n, 5)


def test_network_sampler_converges_to_ode_solution(orc, ode_case):
    w, cond, z = ode_case
    ref = _dop853(orc, w, cond, z)
    errs = [np.abs(orc.sample_raw_rk4(w, cond, K, z) - ref).max() for K in (2, 4, 8, 16)]
    print("rk4 errors", errs)
    # fourth order: each halving of h divides the error by about 16
    for i in range(3):
        assert 13.0 < errs[i] / errs[i + 1] < 19.0
    # at the paper's 12 steps RK4 is far closer to the flow than Euler at the same K
    e12 = np.abs(orc.sample_raw_rk4(w, cond, 12, z) - ref).max()
    assert e12 < 1e-4 * np.abs(orc.sample_raw(w, cond, 12, z) - ref).max()
