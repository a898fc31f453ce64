"""Pins for the oracle's surface source (isotropic incident flux on one side of the domain: the
boundary drive of the paper's second benchmark, "Benchmark Performance").

Each pin is fixed independently of the oracle:
  * pure absorber (c = 0, no collisions): every history is a straight chord from its entry
    point; the escaping weight E[exp(-sigma d)] and the total track length E[(1 - exp(-sigma d))
    / sigma] are integrated here by quadrature over the entry height and sin(theta);
  * pure scattering (c = 1) in a homogeneous square: the mean path of particles entering with
    the cosine law over the whole boundary is pi A / P for every scattering thickness (the
    mean-chord invariance that also pins the single-cell walk); by the square's symmetry
    entering through one side gives the same mean, pi D / 4;
  * rotation covariance: turning the materials, the source cell and its side by a quarter turn
    clockwise turns every tally map the same way, exactly (the transmission of each cell visit
    happens in a canonical frame that the rotation does not change).
"""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs


def _square(n, tau, c, L=1.0, src_face=3, w_min=1e-9):
    t = np.full(n * n, tau, np.float64)
    cc = np.full(n * n, c, np.float64)
    x0, y0, nx_, ny_ = {3: (0, 0, 1, n), 1: (n - 1, 0, 1, n), 0: (0, 0, n, 1), 2: (0, n - 1, n, 1)}[src_face]
    return inputs.Problem(n, n, L, t, cc, x0, y0, nx_, ny_, False, w_min, src_face)


def _chords(D, m=2000):
    """Chord length d(y, s) from (0, y) along (sqrt(1 - s^2), s) across the square [0, D]^2, on a
    midpoint grid of y in (0, D) and s = sin(theta) in (-1, 1) (the cosine law)."""
    y = (np.arange(m) + 0.5) / m * D
    s = (np.arange(m) + 0.5) / m * 2.0 - 1.0
    Y, S = np.meshgrid(y, s, indexing="ij")
    C = np.sqrt(1.0 - S * S)
    with np.errstate(divide="ignore"):
        dy = np.where(S > 0, (D - Y) / S, np.where(S < 0, Y / -S, np.inf))
    return np.minimum(D / C, dy)


@pytest.mark.parametrize("tau_cell", [0.25, 1.0])
def test_pure_absorber_escape_and_track_length_by_quadrature(orc, tau_cell):
    n, L, N = 4, 0.5, 200_000
    prob = _square(n, tau_cell, 0.0, L)
    o = orc.transport(prob, seed=3, h_begin=0, h_end=N, nthreads=8)
    sig = tau_cell / L
    d = _chords(n * L)
    esc = np.exp(-sig * d)
    p_q, p2_q = esc.mean(), (esc ** 2).mean()
    trk_q = ((1.0 - esc) / sig).mean()
    se = math.sqrt((p2_q - p_q ** 2) / N)
    print(f"tau {tau_cell}: escape {o['leak'] / N:.5f} vs {p_q:.5f} (se {se:.1e}); track "
          f"{o['flux'].sum() * L * L / N:.5f} vs {trk_q:.5f}")
    assert abs(o["leak"] / N - p_q) < 4.5 * se
    assert abs(o["leak"] + o["absorbed"].sum() + o["cutoff"] - N) < 1e-9 * N
    # track length: same chords, so its error is of the same relative size
    assert abs(o["flux"].sum() * L * L / N - trk_q) < 4.5 * se / sig


@pytest.mark.parametrize("tau_cell", [0.5, 3.0])
def test_pure_scattering_mean_path_is_pi_d_over_4(orc, tau_cell):
    n, L = 4, 1.0
    prob = _square(n, tau_cell, 1.0, L)
    means = []
    for b in range(16):
        o = orc.transport(prob, seed=5, h_begin=b * 5000, h_end=(b + 1) * 5000, nthreads=8)
        assert abs(o["leak"] - 5000) < 1e-9 * 5000 and o["cutoff"] == 0.0
        means.append(o["flux"].sum() * L * L / 5000)
    m, se = np.mean(means), np.std(means, ddof=1) / math.sqrt(len(means))
    print(f"tau {tau_cell}: E[path] {m:.4f} +- {se:.4f}, pi D / 4 = {math.pi * n * L / 4:.4f}")
    assert abs(m - math.pi * n * L / 4) < 4.5 * se


def _rot_cw(a):
    """Grid array [ny, nx] (row j = y, increasing upwards) turned a quarter turn clockwise,
    (x, y) -> (y, n - x): cell (i, j) moves to (j, n - 1 - i).  (np.rot90 turns the array as
    printed, rows downwards, so its counter-clockwise turn is this clockwise one.)"""
    return np.rot90(a, k=1)


def test_quarter_turns_turn_the_tallies(orc):
    n, j0 = 6, 2
    g = np.random.default_rng(7)
    tau = np.exp(g.uniform(math.log(0.2), math.log(8.0), (n, n)))
    c = g.uniform(0.3, 1.0, (n, n))
    # source cell (0, j0) on the left side; a clockwise quarter turn sends the left side to the
    # top, the top to the right, the right to the bottom
    cell, face = (0, j0), 3
    ref = None
    for r in range(4):
        prob = inputs.Problem(n, n, 1.0, tau.reshape(-1).copy(), c.reshape(-1).copy(), cell[0], cell[1],
                              1, 1, False, 1e-9, face)
        o = orc.transport(prob, seed=11, h_begin=0, h_end=3000, nthreads=4)
        fl = o["flux"].reshape(n, n)
        if ref is None:
            ref = fl
        else:
            ref = _rot_cw(ref)
            np.testing.assert_allclose(fl, ref, rtol=1e-12, atol=1e-12)
        tau, c = _rot_cw(tau), _rot_cw(c)
        # (i, j) -> (j, n - 1 - i); sides 3 -> 2 -> 1 -> 0
        cell = (cell[1], n - 1 - cell[0])
        face = (face - 1) % 4


def test_single_cell_surface_source_mean_chord(orc):
    # one unit cell, no collisions: the cosine-law chord from one side has mean pi / 4
    prob = _square(1, 1e-12, 1.0, 1.0)
    N = 200_000
    o = orc.transport(prob, seed=2, h_begin=0, h_end=N, nthreads=8)
    assert abs(o["leak"] - N) < 1e-9 * N
    # mean chord of a unit square from one side with the cosine law: pi / 4
    assert abs(o["flux"].sum() / N - math.pi / 4) < 4.5 * 0.35 / math.sqrt(N)
