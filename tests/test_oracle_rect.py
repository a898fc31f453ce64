"""Pins for the oracle's walk through a rectangular cell (paper eq. 10: the condition carries
the cell's optical width and height W~ = W sigma, H~ = H sigma; here the canonical cell is
[0, A] x [0, 1] in units of the entry face, A = W / H, tau = sigma_t H).

Each pin is fixed independently of the oracle:
  * no collisions: the exit is the closed-form ray-rectangle intersection;
  * A = 1 is the square walk, bit for bit;
  * cosine-law entry, pure absorber: transmitted fraction E[exp(-tau d)] by chord quadrature;
  * mean-chord invariance over the whole boundary (pi Area / Perimeter for any scattering
    thickness), split by entry side: E(A; tau) + A^2 E(1/A; tau A) = pi A / 2, where E(A; tau)
    is the mean path (units of the entry face) entering a side of length 1 of the A x 1 cell;
  * collisions form a Poisson process along the path: E[n_coll] = tau_s E[path].
"""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs


def _cond(n, tau, c, A, seed):
    b = inputs.fixed_cell_conditions(n, tau, c, seed)
    return inputs.Conditions(b.log_tau, b.c, b.y_in, b.sin_th, np.full(n, np.float32(math.log(A))))


def _ray(y, s, A):
    """Exit of the ray from (0, y) along (sqrt(1 - s^2), s) through [0, A] x [0, 1]: face,
    position (fraction of the face, counter-clockwise) and length."""
    u = np.sqrt(1.0 - s * s)
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = (A - 0.0) / u
        ty = np.where(s > 0, (1.0 - y) / s, np.where(s < 0, -y / s, np.inf))
    xface = tx <= ty
    d = np.where(xface, tx, ty)
    ye = np.clip(y + d * s, 0, 1)
    xe = np.clip(d * u, 0, A)
    face = np.where(xface, 1, np.where(s > 0, 2, 0))
    pos = np.where(face == 1, ye, np.where(face == 2, (A - xe) / A, xe / A))
    return face, pos, d


@pytest.mark.parametrize("A", [0.3, 2.5])
def test_no_collision_exit_is_the_ray_rectangle_intersection(orc, A):
    cond = _cond(20_000, 1e-12, 1.0, A, seed=3)
    o = orc.mc_transmit(cond, 0, seed=1)
    y = cond.y_in.astype(np.float64)
    s = cond.sin_th.astype(np.float64)
    face, pos, d = _ray(y, s, float(np.exp(np.float64(cond.log_aspect[0]))))
    assert np.all(o["ncoll"] == 0)
    np.testing.assert_array_equal(o["face"], face)
    np.testing.assert_allclose(o["pos"], pos, atol=1e-12)
    np.testing.assert_allclose(o["len"], d, rtol=1e-12)


def test_unit_aspect_is_the_square_walk(orc):
    b = inputs.fixed_cell_conditions(5_000, 7.0, 0.9, seed=4)
    r = inputs.Conditions(b.log_tau, b.c, b.y_in, b.sin_th, np.zeros(5_000, np.float32))
    for mode in (0, 1):
        o1, o2 = orc.mc_transmit(b, mode, seed=2), orc.mc_transmit(r, mode, seed=2)
        for k in o1:
            np.testing.assert_array_equal(o1[k], o2[k])


def _chord_quadrature(tau, A, m=4000):
    y = (np.arange(m) + 0.5) / m
    s = (np.arange(m) + 0.5) / m * 2.0 - 1.0
    Y, S = np.meshgrid(y, s, indexing="ij")
    _, _, d = _ray(Y, S, A)
    return float(np.mean(np.exp(-tau * d)))


@pytest.mark.parametrize("tau,A", [(1.0, 0.4), (0.5, 3.0)])
def test_pure_absorber_escape_by_quadrature(orc, tau, A):
    n = 200_000
    o = orc.mc_transmit(_cond(n, tau, 0.0, A, seed=5), 1, seed=3, nthreads=8)
    p_mc = np.mean(o["face"] >= 0)
    p_q = _chord_quadrature(tau, A)
    se = math.sqrt(p_q * (1 - p_q) / n)
    print(f"tau {tau} A {A}: escape {p_mc:.5f} vs {p_q:.5f}")
    assert abs(p_mc - p_q) < 4.5 * se


@pytest.mark.parametrize("tau,A", [(0.5, 0.5), (4.0, 2.0), (10.0, 0.25)])
def test_mean_chord_invariance_split_by_entry_side(orc, tau, A):
    n = 100_000
    a = orc.mc_transmit(_cond(n, tau, 1.0, A, seed=6), 0, seed=4, nthreads=8)["len"]
    b = orc.mc_transmit(_cond(n, tau * A, 1.0, 1.0 / A, seed=7), 0, seed=5, nthreads=8)["len"]
    lhs = a.mean() + A * A * b.mean()
    se = math.sqrt(a.var() / n + A ** 4 * b.var() / n)
    print(f"tau {tau} A {A}: E(A) + A^2 E(1/A) = {lhs:.4f} +- {se:.4f} vs pi A / 2 = {math.pi * A / 2:.4f}")
    assert abs(lhs - math.pi * A / 2) < 4.5 * se


@pytest.mark.parametrize("A", [0.5, 3.0])
def test_collisions_per_unit_length(orc, A):
    n, tau_s = 100_000, 3.0
    o = orc.mc_transmit(_cond(n, tau_s, 1.0, A, seed=8), 0, seed=6, nthreads=8)
    diff = o["ncoll"].astype(np.float64) - tau_s * o["len"]
    assert abs(diff.mean()) < 4.5 * diff.std() / math.sqrt(n)


def test_rectangular_condition_features(orc):
    c = inputs.transmission_conditions(6, seed=9, log_aspect_range=(-1.0, 1.0))
    f = orc.condition_features(c)
    assert f.shape == (6, 5)
    np.testing.assert_allclose(f[:, 4], c.log_aspect)
    sq = inputs.transmission_conditions(6, seed=9)
    np.testing.assert_array_equal(orc.condition_features(sq), f[:, :4])
