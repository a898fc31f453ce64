"""GPU transport with a surface source (isotropic incident flux on one side of the domain: the
drive of the paper's second benchmark, "Benchmark Performance") against the FP64 oracle, and
the rotation covariance that pins the source's direction conventions on the oracle side.

As in test_gpu_transport.py, the analog sampler draws the same Philox words as the oracle for
every history, so flux maps agree far inside their statistical error (bar 5e-5 relative L1).
"""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _run(binding, prob, n, seed, sampler, model=None, K=16, capacity=1 << 18):
    from paper_2512_13965_amd import transport
    w = binding.World(capacity, 2, max(prob.n_cells, 1 << 12))
    out = transport.run_problem(w, prob, n, seed, sampler, model, K)
    w.close()
    return out


def _side_problem(n, face, seed):
    g = np.random.default_rng(seed)
    tau = np.exp(g.uniform(math.log(0.2), math.log(6.0), n * n))
    c = g.uniform(0.3, 1.0, n * n)
    x0, y0, snx, sny = {3: (0, 1, 1, n - 2), 1: (n - 1, 0, 1, n), 0: (1, 0, n - 1, 1), 2: (0, n - 1, n, 1)}[face]
    return inputs.Problem(n, n, 0.8, tau, c, x0, y0, snx, sny, False, 1e-6, face)


@pytest.mark.parametrize("name,prob", [("hohlraum16", inputs.hohlraum_problem(16))] +
                         [(f"side{f}", _side_problem(5, f, 30 + f)) for f in range(4)])
def test_surface_source_mc_transport_matches_oracle(orc, name, prob):
    binding = require_gpu()
    n = 20_000
    g = _run(binding, prob, n, 13, binding.SAMPLER_MC)
    o = orc.transport(prob, seed=13, h_begin=0, h_end=n, nthreads=8)
    rel = np.abs(g["flux"] - o["flux"]).sum() / np.abs(o["flux"]).sum()
    print(f"{name}: flux L1 rel diff {rel:.2e}; leak {g['leak'].sum():.4f} vs {o['leak']:.4f}; "
          f"transmissions {g['transmissions']} vs {o['events']:.0f}")
    assert rel < 5e-5
    assert abs(g["leak"].sum() - o["leak"]) < 1e-4 * n
    assert abs(g["absorbed"].sum() + g["leak"].sum() + g["cutoff"].sum() - n) < 1e-9 * n


def test_quarter_turns_turn_the_gpu_tallies():
    # the oracle-side pin (test_oracle_surface.py) on the GPU path: materials, source cell and
    # side turned a quarter turn clockwise turn the flux map the same way
    binding = require_gpu()
    n = 6
    g = np.random.default_rng(8)
    tau = np.exp(g.uniform(math.log(0.2), math.log(8.0), (n, n)))
    c = g.uniform(0.3, 1.0, (n, n))
    cell, face, ref = (0, 2), 3, None
    for r in range(4):
        prob = inputs.Problem(n, n, 1.0, tau.reshape(-1).copy(), c.reshape(-1).copy(), cell[0], cell[1],
                              1, 1, False, 1e-9, face)
        fl = _run(binding, prob, 20_000, 11, binding.SAMPLER_MC)["flux"].reshape(n, n)
        if ref is None:
            ref = fl
        else:
            ref = np.rot90(ref, k=1)          # clockwise for rows that grow upwards
            np.testing.assert_allclose(fl, ref, rtol=1e-9, atol=1e-9)
        tau, c = np.rot90(tau, k=1), np.rot90(c, k=1)
        cell = (cell[1], n - 1 - cell[0])
        face = (face - 1) % 4


def test_surface_problem_alone_and_in_mix_agree():
    binding = require_gpu()
    from paper_2512_13965_amd import transport
    a = inputs.hohlraum_problem(16)
    b = inputs.lattice_problem(2)
    na, nb = 20_000, 20_000
    w = binding.World(1 << 17, 4, 1 << 12)
    alone = transport.run_problem(w, a, na, 21, binding.SAMPLER_MC)
    pb = w.add_problem(b, 99)
    pa = w.add_problem(a, 21)
    w.inject(pb, 0, nb)
    w.inject(pa, 0, na)
    alive = 1
    while alive:
        alive = w.step(binding.SAMPLER_MC)
    mix = w.tally(pa)
    w.close()
    for k in ("flux", "absorbed", "leak", "cutoff"):
        np.testing.assert_allclose(mix[k], alone[k], rtol=1e-12, atol=1e-12 * na)


def test_surface_source_descriptor_errors():
    binding = require_gpu()
    w = binding.World(1000, 2, 1000)
    base = _side_problem(5, 3, 1)
    bad = [
        dict(src_face=4),
        dict(src_face=-2),
        dict(src_x0=1),                         # left strip must start at x = 0
        dict(src_nx=2),                         # and be one cell wide
        dict(reflect=True),                     # surface sources need vacuum boundaries
    ]
    for change in bad:
        p = inputs.Problem(**{**base.__dict__, **change})
        with pytest.raises(binding.GmcError):
            w.add_problem(p, 1)
    w.close()
