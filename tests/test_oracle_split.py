"""Pins for the oracle's first-flight split (an analytic variant beside the paper's single
model: a transmission that meets no collision is placed exactly, and only collided ones are
left to a model fitted on collided exits).

Each pin is fixed independently of the oracle's split code:
  * the uncollided fraction of a cell equals the fraction of analog walks with no collision
    (the walk draws other random numbers: a statistical comparison);
  * for a pure absorber in analog mode the escape probability is the same mean, E[exp(-tau d)],
    integrated by quadrature (P2's integral), which the uncollided fraction must match at c = 1;
  * uncollided exits are the ray's exits: closed-form face, position and length.
"""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs


@pytest.mark.parametrize("tau", [0.1, 1.0, 4.0])
def test_uncollided_fraction_is_the_no_collision_fraction_of_the_walk(orc, tau):
    n = 200_000
    cond = inputs.fixed_cell_conditions(n, tau, 1.0, seed=11)
    sp = orc.uncollided_split(cond, seed=3)
    wk = orc.mc_transmit(cond, 0, seed=4, nthreads=8)
    p_s, p_w = sp["flag"].mean(), (wk["ncoll"] == 0).mean()
    se = math.sqrt(p_w * (1 - p_w) * 2 / n)
    print(f"tau {tau}: uncollided {p_s:.5f} vs walk {p_w:.5f}")
    assert abs(p_s - p_w) < 4.5 * se


def test_uncollided_fraction_by_quadrature(orc):
    tau, n = 1.0, 400_000
    cond = inputs.fixed_cell_conditions(n, tau, 1.0, seed=12)
    p_s = orc.uncollided_split(cond, seed=5)["flag"].mean()
    m = 2000
    y = (np.arange(m) + 0.5) / m
    s = (np.arange(m) + 0.5) / m * 2 - 1
    Y, S = np.meshgrid(y, s, indexing="ij")
    U = np.sqrt(1 - S * S)
    with np.errstate(divide="ignore"):
        ty = np.where(S > 0, (1 - Y) / S, np.where(S < 0, -Y / S, np.inf))
    d = np.minimum(1.0 / U, ty)
    p_q = float(np.mean(np.exp(-tau * d)))
    assert abs(p_s - p_q) < 4.5 * math.sqrt(p_q * (1 - p_q) / n)


def test_uncollided_exits_are_ray_exits_and_xy_keeps_the_direction(orc):
    c = inputs.xy_conditions(5_000, seed=13)
    sp = orc.uncollided_split(c, seed=6)
    u, v, y = c.omega_x.astype(np.float64), c.sin_th.astype(np.float64), c.y_in.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        tx, ty = 1.0 / u, np.where(v > 0, (1 - y) / v, np.where(v < 0, -y / v, np.inf))
    np.testing.assert_allclose(sp["len"], np.minimum(tx, ty), rtol=1e-12)
    np.testing.assert_array_equal(sp["face"], np.where(tx <= ty, 1, np.where(v > 0, 2, 0)))
    np.testing.assert_array_equal(sp["u"], u)
    np.testing.assert_array_equal(sp["v"], v)


@pytest.mark.parametrize("tau,c", [(0.3, 1.0), (2.0, 0.5), (5.0, 0.2)])
def test_normal_incidence_uncollided_fraction_is_exp_minus_c_tau(orc, tau, c):
    # entering along the normal, every ray crosses the unit cell in d_b = 1: the uncollided
    # fraction is exp(-c tau) (flights of rate c tau, eq. 4) and every uncollided exit is the
    # opposite face at the entry height
    n = 200_000
    cond = inputs.fixed_cell_conditions(n, tau, c, seed=14)
    cond.sin_th[:] = 0.0
    sp = orc.uncollided_split(cond, seed=7)
    p = math.exp(-c * tau)
    assert abs(sp["flag"].mean() - p) < 4.5 * math.sqrt(p * (1 - p) / n)
    np.testing.assert_array_equal(sp["face"], 1)
    np.testing.assert_allclose(sp["pos"], cond.y_in.astype(np.float64), atol=1e-7)
    np.testing.assert_allclose(sp["len"], 1.0, rtol=1e-12)
