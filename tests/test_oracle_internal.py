"""Pins for the oracle's walk started inside the cell (the walk the internal, volumetric-source
model replaces; paper "Network Architecture and Inputs": the internal model's condition is the
two-dimensional birth position and the birth direction) and for its network input layout.

Each pin is fixed independently of the oracle:
  * with no collisions the exit is the ray-box intersection, computed here in closed form;
  * a uniform birth position with an isotropic direction exits each face with probability 1/4;
  * a pure absorber (analog mode, c = 0) lets a birth escape with probability E[exp(-tau d)],
    d the distance to the boundary along the birth direction, integrated here by quadrature;
  * collisions along a pure-scattering path form a Poisson process of rate tau_s per unit
    length, so E[n_coll] = tau_s E[path];
  * a birth on the left face pointing into the cell is the boundary walk of the same stream.
"""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs


def _ray_exit(x, y, u, v):
    """Closed-form exit of the ray (x, y) + s (u, v) from the unit square: face, position along it
    (counter-clockwise: bottom x, right y, top 1 - x, left 1 - y) and distance."""
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = np.where(u > 0, (1 - x) / u, np.where(u < 0, -x / u, np.inf))
        ty = np.where(v > 0, (1 - y) / v, np.where(v < 0, -y / v, np.inf))
    xface = tx <= ty
    d = np.where(xface, tx, ty)
    ye = np.clip(y + d * v, 0, 1)
    xe = np.clip(x + d * u, 0, 1)
    face = np.where(xface, np.where(u > 0, 1, 3), np.where(v > 0, 2, 0))
    pos = np.where(face == 1, ye, np.where(face == 3, 1 - ye, np.where(face == 2, 1 - xe, xe)))
    return face, pos, d


def _f64(c):
    return tuple(np.asarray(a, np.float64) for a in (c.x, c.y, c.cos_phi, c.sin_phi))


def test_no_collision_walk_is_the_ray_box_exit(orc):
    cond = inputs.fixed_internal_conditions(20_000, 1e-12, 1.0, seed=5)
    o = orc.mc_transmit_internal(cond, 0, seed=1)
    face, pos, d = _ray_exit(*_f64(cond))
    assert np.all(o["ncoll"] == 0)
    np.testing.assert_array_equal(o["face"], face)
    np.testing.assert_allclose(o["pos"], pos, atol=1e-12)
    np.testing.assert_allclose(o["len"], d, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(o["u"], np.asarray(cond.cos_phi, np.float64), rtol=0, atol=0)


@pytest.mark.parametrize("tau", [1.0, 10.0])
def test_uniform_isotropic_births_exit_each_face_a_quarter(orc, tau):
    n = 200_000
    cond = inputs.fixed_internal_conditions(n, tau, 1.0, seed=6)
    o = orc.mc_transmit_internal(cond, 0, seed=2, nthreads=8)
    frac = np.bincount(o["face"], minlength=4) / n
    sig = math.sqrt(0.25 * 0.75 / n)
    assert np.all(np.abs(frac - 0.25) < 4.5 * sig), frac


def _escape_quadrature(tau, m=160, mphi=720):
    """E[exp(-tau d)] over a uniform birth point and an isotropic direction (midpoint rule)."""
    g = (np.arange(m) + 0.5) / m
    phi = (np.arange(mphi) + 0.5) * 2 * math.pi / mphi
    X, Y, P = np.meshgrid(g, g, phi, indexing="ij")
    _, _, d = _ray_exit(X.ravel(), Y.ravel(), np.cos(P).ravel(), np.sin(P).ravel())
    return float(np.mean(np.exp(-tau * d))), float(np.mean(d))


@pytest.mark.parametrize("tau", [0.5, 2.0])
def test_pure_absorber_escape_probability(orc, tau):
    n = 200_000
    cond = inputs.fixed_internal_conditions(n, tau, 0.0, seed=7)
    o = orc.mc_transmit_internal(cond, 1, seed=3, nthreads=8)
    p_mc = np.mean(o["face"] >= 0)
    p_q, _ = _escape_quadrature(tau)
    sig = math.sqrt(p_q * (1 - p_q) / n)
    print(f"tau {tau}: escape MC {p_mc:.5f} quadrature {p_q:.5f}")
    assert abs(p_mc - p_q) < 4.5 * sig
    assert np.all(o["face"] >= -1) and np.all(o["ncoll"][o["face"] >= 0] == 0)


def test_mean_distance_to_the_boundary(orc):
    # tau -> 0: the mean path is the mean distance from a uniform point to the boundary along an
    # isotropic direction
    cond = inputs.fixed_internal_conditions(400_000, 1e-12, 1.0, seed=8)
    o = orc.mc_transmit_internal(cond, 0, seed=4, nthreads=8)
    _, d_q = _escape_quadrature(0.0)
    se = o["len"].std() / math.sqrt(len(cond))
    assert abs(o["len"].mean() - d_q) < 4.5 * se


@pytest.mark.parametrize("tau_s", [2.0, 20.0])
def test_collisions_per_unit_length(orc, tau_s):
    n = 100_000
    cond = inputs.fixed_internal_conditions(n, tau_s, 1.0, seed=9)
    o = orc.mc_transmit_internal(cond, 0, seed=5, nthreads=8)
    diff = o["ncoll"].astype(np.float64) - tau_s * o["len"]
    assert abs(diff.mean()) < 4.5 * diff.std() / math.sqrt(n)


def test_left_face_birth_is_the_boundary_walk(orc):
    n = 5_000
    b = inputs.fixed_cell_conditions(n, 5.0, 0.8, seed=10)
    cos_th = np.sqrt(1.0 - b.sin_th.astype(np.float64) ** 2).astype(np.float32)
    ic = inputs.InternalConditions(b.log_tau, b.c, np.zeros(n, np.float32), b.y_in, cos_th, b.sin_th)
    for mode in (0, 1):
        o_b = orc.mc_transmit(b, mode, seed=6)
        o_i = orc.mc_transmit_internal(ic, mode, seed=6)
        # same Philox words, same collisions; the birth direction's cosine is rounded to float32
        # in the internal condition, so continuous outputs agree to that rounding
        np.testing.assert_array_equal(o_b["face"], o_i["face"])
        np.testing.assert_array_equal(o_b["ncoll"], o_i["ncoll"])
        for k in ("pos", "u", "v", "len"):
            np.testing.assert_allclose(o_b[k], o_i[k], rtol=1e-5, atol=1e-6)


def test_internal_condition_feature_order(orc):
    c = inputs.internal_conditions(4, seed=11)
    f = orc.condition_features(c)
    assert f.shape == (4, 6)
    np.testing.assert_allclose(f[:, 0], c.log_tau)
    np.testing.assert_allclose(f[:, 1], c.c)
    np.testing.assert_allclose(f[:, 2], 2.0 * c.x.astype(np.float64) - 1.0)
    np.testing.assert_allclose(f[:, 3], 2.0 * c.y.astype(np.float64) - 1.0)
    np.testing.assert_allclose(f[:, 4], c.cos_phi)
    np.testing.assert_allclose(f[:, 5], c.sin_phi)


def test_internal_network_input_is_x_t_condition(orc):
    # the first layer sees [x0..x4, t, condition]: a network whose first layer reads only column
    # 6 + j returns a function of feature j alone
    c = inputs.internal_conditions(8, seed=13)
    f = orc.condition_features(c)
    for j in range(6):
        ww = inputs.random_weights(16, seed=12, n_in=inputs.N_IN_INTERNAL)
        ww.W[0][:] = 0.0
        ww.W[0][:, 6 + j] = 1.0
        x = np.zeros((8, 5))
        v = orc.velocity(ww, x, 0.3, f)
        # same feature value -> same output; the map is monotone in the feature (SiLU chain)
        ref = orc.velocity(ww, x, 0.3, np.repeat(f[:1], 8, axis=0))
        same = np.isclose(f[:, j], f[0, j])
        np.testing.assert_allclose(v[same], ref[same])
        assert not np.allclose(v[~same], ref[~same])
