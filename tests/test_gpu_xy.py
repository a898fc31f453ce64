"""GPU parity in XY geometry (paper eq. 1 over the sphere, the problem invariant along z):
the analog walk with projected spherical directions, and transport with volumetric and surface
sources, each against the FP64 oracle on the same Philox streams.  Tolerances are those of the
flatland tests (test_gpu_walk.py, test_gpu_transport.py)."""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu
from tests.test_gpu_walk import _compare, _gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1])
def test_xy_walk_matches_oracle(orc, mode):
    binding = require_gpu()
    cond = inputs.xy_conditions(100_003, seed=71, c_range=(0.5, 1.0))
    g = _gpu(binding, cond, mode, seed=8)
    o = orc.mc_transmit(cond, mode, seed=8, nthreads=8)
    _compare(g, o, max_mismatch=5e-4)
    assert np.all(g["dir_cos"] ** 2 + g["dir_sin"] ** 2 <= 1.0 + 1e-5)


def test_xy_walk_rectangular_cells_match_oracle(orc):
    binding = require_gpu()
    c = inputs.xy_conditions(50_000, seed=72)
    la = np.random.default_rng(3).uniform(math.log(0.25), math.log(4.0), len(c)).astype(np.float32)
    cond = inputs.Conditions(c.log_tau, c.c, c.y_in, c.sin_th, la, c.omega_x)
    _compare(_gpu(binding, cond, 0, seed=9), orc.mc_transmit(cond, 0, seed=9, nthreads=8), max_mismatch=5e-4)


def test_xy_mean_path_is_four_area_over_perimeter():
    binding = require_gpu()
    for tau in (1.0, 30.0):
        g = _gpu(binding, inputs.fixed_xy_conditions(400_000, tau, 1.0, seed=5), 0, seed=3)
        se = g["path"].std() / math.sqrt(len(g["path"]))
        assert abs(g["path"].mean() - 1.0) < 4.5 * se


def _xy_problem(Ly, face, seed):
    g = np.random.default_rng(seed)
    n = 5
    tau = np.exp(g.uniform(math.log(0.2), math.log(6.0), n * n))
    c = g.uniform(0.3, 1.0, n * n)
    if face < 0:
        return inputs.Problem(n, n, 0.8, tau, c, 1, 2, 3, 2, False, 1e-6, -1, Ly, True)
    return inputs.Problem(n, n, 0.8, tau, c, 0, 0, 1, n, False, 1e-6, 3, Ly, True)


@pytest.mark.parametrize("Ly,face", [(0.0, -1), (0.0, 3), (0.4, -1), (1.5, 3)])
def test_xy_mc_transport_matches_oracle(orc, Ly, face):
    binding = require_gpu()
    from paper_2512_13965_amd import transport
    prob = _xy_problem(Ly, face, 80)
    n = 20_000
    w = binding.World(1 << 17, 1, 1 << 12)
    g = transport.run_problem(w, prob, n, 19, binding.SAMPLER_MC)
    w.close()
    o = orc.transport(prob, seed=19, h_begin=0, h_end=n, nthreads=8)
    rel = np.abs(g["flux"] - o["flux"]).sum() / np.abs(o["flux"]).sum()
    print(f"XY Ly {Ly} face {face}: flux L1 {rel:.2e}, leak {g['leak'].sum():.4f} vs {o['leak']:.4f}")
    assert rel < 5e-5
    assert abs(g["absorbed"].sum() + g["leak"].sum() + g["cutoff"].sum() - n) < 1e-9 * n


def test_xy_world_geometry_checks():
    binding = require_gpu()
    w = binding.World(1 << 12, 2, 1 << 10)
    w.add_problem(_xy_problem(0.0, -1, 1), 1)
    flat = inputs.checkerboard_problem(4, src=2)
    with pytest.raises(binding.GmcError):
        w.add_problem(flat, 2)                                   # one geometry per world
    m = binding.Model(inputs.pack_blob(inputs.random_weights(128, 1)), "fp32")
    with pytest.raises(binding.GmcError):
        w.step(binding.SAMPLER_GMC, m, 4)                        # flatland model, XY world
    w.close()
    m.close()
