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


@pytest.mark.parametrize("prec,H,K", [("fp32", 256, 16), ("bf16", 512, 16)])
def test_xy_sampler_matches_oracle(orc, prec, H, K):
    # an XY-geometry boundary model (11 inputs, flag bit 0): condition (ln tau, c, 2 y - 1,
    # omega_y, omega_x); exits decoded into the unit disk
    import torch
    binding = require_gpu()
    n = 20_011
    cond = inputs.xy_conditions(n, seed=73)
    w = inputs.random_weights(H, 6, n_in=inputs.N_IN_RECT, flags=1)
    m = binding.Model(inputs.pack_blob(w), prec)
    raw = torch.empty(5 * n, dtype=torch.float32, device="cuda")
    out = binding.gmc_sample(m, binding.DeviceCond.from_host(cond), "euler", K, 2, 0, raw=raw).to_host()
    torch.cuda.synchronize()
    m.close()
    raw = raw.view(5, n).cpu().numpy().astype(np.float64)
    from tests.gpu_util import sample_indices
    idx = sample_indices(n, 200, seed=5)
    z = np.stack([orc.noise(2, int(i), 1)[:, 0] for i in idx], axis=1)
    ref = orc.sample_raw(w, cond.subset(idx), K, z, orc.PREC_FP64 if prec == "fp32" else orc.PREC_BF16_EXP2)
    err = np.abs(raw[:, idx].T - ref).max(axis=1)
    print(f"XY {prec}: p99 {np.quantile(err, .99):.2e} max {err.max():.2e}")
    tol = (1e-5, 1e-5) if prec == "fp32" else (1e-5, 5e-5)
    assert np.quantile(err, 0.99) < tol[0] and err.max() < tol[1]
    # the kernel's decoder against the oracle's XY decoder on the kernel's own raw output
    d = orc.decode(raw.T, xy=True)
    np.testing.assert_array_equal(out["face"], d["face"])
    np.testing.assert_allclose(out["dir_cos"], d["u"], atol=2e-6)
    np.testing.assert_allclose(out["dir_sin"], d["v"], atol=2e-6)
    assert np.all(out["dir_cos"] ** 2 + out["dir_sin"] ** 2 <= 1.0 + 1e-5)


def test_xy_model_checks():
    binding = require_gpu()
    with pytest.raises(binding.GmcError):
        binding.Model(inputs.pack_blob(inputs.random_weights(128, 1, flags=1)), "fp32")   # XY needs 11 inputs
    mxy = binding.Model(inputs.pack_blob(inputs.random_weights(128, 1, n_in=11, flags=1)), "fp32")
    flat = binding.DeviceCond.from_host(inputs.transmission_conditions(64, 1))
    with pytest.raises(binding.GmcError):
        binding.gmc_sample(mxy, flat, "euler", 4, 0)                 # XY model needs omega_x
    w = binding.World(1 << 12, 1, 1 << 10)
    w.add_problem(inputs.checkerboard_problem(4, src=2), 1)
    with pytest.raises(binding.GmcError):
        w.step(binding.SAMPLER_GMC, mxy, 4)                          # XY model, flatland world
    w.close()
    mxy.close()


def test_xy_gmc_transport_balances():
    binding = require_gpu()
    from paper_2512_13965_amd import transport
    m = binding.Model(inputs.pack_blob(inputs.random_weights(256, 3, n_in=11, flags=1)), "bf16")
    w = binding.World(1 << 16, 1, 1 << 12)
    for face in (-1, 3):
        r = transport.run_problem(w, _xy_problem(0.0, face, 81), 10_000, 5, binding.SAMPLER_GMC, m, 8)
        assert abs(r["absorbed"].sum() + r["leak"].sum() + r["cutoff"].sum() - 10_000) < 1e-6
    w.close()
    m.close()
