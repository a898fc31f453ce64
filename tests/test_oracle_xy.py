"""Pins for the oracle's walk in XY geometry (paper eq. 1 integrates over the sphere, and the
condition's direction lives in the unit disk of direction cosines: the problem is invariant
along z and a particle's in-plane direction is the projection of a unit direction).

Each pin is fixed independently of the oracle:
  * no collisions: the exit is the closed-form ray-square intersection along the projected
    direction, the path being the three-dimensional length;
  * isotropic incident flux on one side of the unit square, pure scattering: the mean
    three-dimensional path is 4 Area / Perimeter = 1 for every scattering thickness (Cauchy's
    mean chord in three dimensions, which scattering leaves unchanged; one side equals the whole
    boundary by symmetry);
  * collisions form a Poisson process along the three-dimensional path: E[n_coll] = tau_s E[l];
  * pure absorber: escape probability E[exp(-tau d)] by quadrature over the entry height, the
    cosine to the normal and the azimuth;
  * the projected entry directions of isotropic incident flux: |omega| <= 1, omega_x > 0, and
    E[omega_x] = 2/3 (the mean cosine of the three-dimensional cosine law).
"""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs


def _ray(y, u, v):
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = 1.0 / u
        ty = np.where(v > 0, (1.0 - y) / v, np.where(v < 0, -y / v, np.inf))
    xface = tx <= ty
    d = np.where(xface, tx, ty)
    ye = np.clip(y + d * v, 0, 1)
    xe = np.clip(d * u, 0, 1)
    face = np.where(xface, 1, np.where(v > 0, 2, 0))
    pos = np.where(face == 1, ye, np.where(face == 2, 1 - xe, xe))
    return face, pos, d


def test_entry_directions_of_isotropic_incident_flux():
    c = inputs.fixed_xy_conditions(400_000, 1.0, 1.0, seed=1)
    ox, oy = c.omega_x.astype(np.float64), c.sin_th.astype(np.float64)
    assert np.all(ox > 0) and np.all(ox * ox + oy * oy <= 1.0 + 1e-6)
    assert abs(ox.mean() - 2.0 / 3.0) < 4.5 * ox.std() / math.sqrt(len(ox))
    assert abs(oy.mean()) < 4.5 * oy.std() / math.sqrt(len(oy))


def test_no_collision_exit_is_the_projected_ray_intersection(orc):
    c = inputs.fixed_xy_conditions(20_000, 1e-12, 1.0, seed=2)
    o = orc.mc_transmit(c, 0, seed=1)
    face, pos, d = _ray(c.y_in.astype(np.float64), c.omega_x.astype(np.float64), c.sin_th.astype(np.float64))
    assert np.all(o["ncoll"] == 0)
    np.testing.assert_array_equal(o["face"], face)
    np.testing.assert_allclose(o["pos"], pos, atol=1e-12)
    np.testing.assert_allclose(o["len"], d, rtol=1e-12)


@pytest.mark.parametrize("tau", [1e-12, 1.0, 10.0, 30.0])
def test_mean_path_is_four_area_over_perimeter(orc, tau):
    n = 200_000
    o = orc.mc_transmit(inputs.fixed_xy_conditions(n, tau, 1.0, seed=3), 0, seed=2, nthreads=8)
    se = o["len"].std() / math.sqrt(n)
    print(f"tau {tau}: E[l] = {o['len'].mean():.4f} +- {se:.4f}")
    assert abs(o["len"].mean() - 1.0) < 4.5 * se


def test_collisions_per_unit_length(orc):
    n, tau_s = 100_000, 4.0
    o = orc.mc_transmit(inputs.fixed_xy_conditions(n, tau_s, 1.0, seed=4), 0, seed=3, nthreads=8)
    diff = o["ncoll"].astype(np.float64) - tau_s * o["len"]
    assert abs(diff.mean()) < 4.5 * diff.std() / math.sqrt(n)


def test_pure_absorber_escape_by_quadrature(orc):
    tau, n = 1.5, 200_000
    o = orc.mc_transmit(inputs.fixed_xy_conditions(n, tau, 0.0, seed=5), 1, seed=4, nthreads=8)
    m = 160
    g = (np.arange(m) + 0.5) / m
    Y, XI, PS = np.meshgrid(g, g, g * 2 * math.pi, indexing="ij")
    _, _, d = _ray(Y.ravel(), np.sqrt(XI.ravel()), np.sqrt(1 - XI.ravel()) * np.cos(PS.ravel()))
    p_q = float(np.mean(np.exp(-tau * d)))
    p_mc = np.mean(o["face"] >= 0)
    se = math.sqrt(p_q * (1 - p_q) / n)
    print(f"escape {p_mc:.5f} vs {p_q:.5f}")
    assert abs(p_mc - p_q) < 4.5 * se


def test_xy_decoding_keeps_projected_directions_inside_the_disk(orc):
    # a4 = -0.5 reaches only the threshold -1: face 1 (right side, outward normal +x)
    raw = np.array([[0.0, 0.3, 0.4, 0.0, -0.5],     # norm 0.5, outward: kept as is
                    [0.0, 1.2, 1.6, 0.0, -0.5],     # norm 2: scaled to norm 1
                    [0.0, -0.3, 0.4, 0.0, -0.5]])   # points inward: x component reflected
    d = orc.decode(raw, xy=True)
    np.testing.assert_array_equal(d["face"], [1, 1, 1])
    np.testing.assert_allclose(np.stack([d["u"], d["v"]], 1), [[0.3, 0.4], [0.6, 0.8], [0.3, 0.4]], atol=1e-15)
    flat = orc.decode(raw)
    np.testing.assert_allclose(np.hypot(flat["u"], flat["v"]), 1.0, atol=1e-15)


def test_xy_condition_features_and_blob_flags(orc):
    c = inputs.xy_conditions(5, seed=6)
    f = orc.condition_features(c)
    assert f.shape == (5, 5)
    np.testing.assert_allclose(f[:, 3], c.sin_th)
    np.testing.assert_allclose(f[:, 4], c.omega_x)
    w = inputs.random_weights(16, 1, n_in=inputs.N_IN_RECT, flags=1)
    back = inputs.unpack_blob(inputs.pack_blob(w))
    assert back.flags == 1 and back.n_in == inputs.N_IN_RECT
