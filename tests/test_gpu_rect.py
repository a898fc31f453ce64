"""GPU parity for rectangular cells (paper eq. 10: the condition carries the optical width and
height): the analog walk through [0, A] x [0, 1], the generative sampler with an 11-input
boundary model (condition ln tau, c, 2 y_in - 1, sin th, ln A), and transport over grids of
rectangular cells, each against the FP64 oracle on the same seeded inputs.

Tolerances are those of the square-cell tests (test_gpu_walk.py, test_gpu_sampler.py,
test_gpu_transport.py)."""
import math

import numpy as np
import pytest
import torch

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu, sample_indices
from tests.test_gpu_walk import _compare, _gpu

pytestmark = pytest.mark.gpu
LA = (math.log(0.25), math.log(4.0))


@pytest.mark.parametrize("mode", [0, 1])
def test_rect_walk_matches_oracle(orc, mode):
    binding = require_gpu()
    cond = inputs.transmission_conditions(100_003, seed=51, c_range=(0.5, 1.0), log_aspect_range=LA)
    g = _gpu(binding, cond, mode, seed=7)
    o = orc.mc_transmit(cond, mode, seed=7, nthreads=8)
    _compare(g, o, max_mismatch=5e-4)


def test_rect_walk_unit_aspect_is_bitwise_the_square_walk():
    binding = require_gpu()
    sq = inputs.transmission_conditions(30_000, seed=52)
    r = inputs.Conditions(sq.log_tau, sq.c, sq.y_in, sq.sin_th, np.zeros(len(sq), np.float32))
    a, b = _gpu(binding, sq, 0, seed=3), _gpu(binding, r, 0, seed=3)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def _sample(binding, w, prec, cond, K, integ="euler", seed=2):
    m = binding.Model(inputs.pack_blob(w), prec)
    assert m.n_in == 11
    dc = binding.DeviceCond.from_host(cond)
    n = len(cond)
    raw = torch.empty(5 * n, dtype=torch.float32, device="cuda")
    out = binding.gmc_sample(m, dc, integ, K, seed, 0, raw=raw)
    torch.cuda.synchronize()
    m.close()
    return raw.view(5, n).cpu().numpy().astype(np.float64), out.to_host()


@pytest.mark.parametrize("prec,H,K", [("fp32", 256, 16), ("bf16", 512, 16), ("fp8", 512, 8)])
def test_rect_sampler_matches_oracle(orc, prec, H, K):
    binding = require_gpu()
    n = 20_011
    cond = inputs.transmission_conditions(n, seed=53, log_aspect_range=LA)
    w = inputs.random_weights(H, 5, n_in=11)
    raw, _ = _sample(binding, w, prec, cond, K)
    idx = sample_indices(n, 200, seed=4)
    z = np.stack([orc.noise(2, int(i), 1)[:, 0] for i in idx], axis=1)
    oprec = {"fp32": orc.PREC_FP64, "bf16": orc.PREC_BF16_EXP2, "fp8": orc.PREC_FP8_EXP2}[prec]
    ref = orc.sample_raw(w, cond.subset(idx), K, z, oprec)
    err = np.abs(raw[:, idx].T - ref).max(axis=1)
    print(f"rect {prec} H={H} K={K}: p99 {np.quantile(err, .99):.2e} max {err.max():.2e}")
    tol = {"fp32": (1e-5, 1e-5), "bf16": (1e-5, 5e-5), "fp8": (1e-4, 3e-4)}[prec]
    assert np.quantile(err, 0.99) < tol[0] and err.max() < tol[1]


def test_rect_model_kind_checks():
    binding = require_gpu()
    m10 = binding.Model(inputs.pack_blob(inputs.random_weights(128, 1)), "fp32")
    cond = binding.DeviceCond.from_host(inputs.transmission_conditions(64, 1, log_aspect_range=LA))
    with pytest.raises(binding.GmcError):
        binding.gmc_sample(m10, cond, "euler", 4, 0)            # square model, aspect given
    w = binding.World(1 << 12, 1, 1 << 10)
    t = np.full(16, 1.0)
    w.add_problem(inputs.Problem(4, 4, 1.0, t, t * 0.9, 1, 1, 2, 2, Ly=0.5), 1)
    with pytest.raises(binding.GmcError):
        w.step(binding.SAMPLER_GMC, m10, 4)                     # rectangular cells, square model
    w.close()
    w = binding.World(1 << 12, 1, 1 << 10)
    with pytest.raises(binding.GmcError):
        w.add_problem(inputs.Problem(4, 4, 1.0, t, t * 0.9, 1, 1, 2, 2, Ly=-1.0), 1)
    w.close()
    m10.close()


def _rect_problem(Ly, face, seed):
    g = np.random.default_rng(seed)
    n = 5
    tau = np.exp(g.uniform(math.log(0.2), math.log(6.0), n * n))
    c = g.uniform(0.3, 1.0, n * n)
    if face < 0:
        return inputs.Problem(n, n, 0.8, tau, c, 1, 2, 3, 2, False, 1e-6, -1, Ly)
    return inputs.Problem(n, n, 0.8, tau, c, 0, 0, 1, n, False, 1e-6, 3, Ly)


@pytest.mark.parametrize("Ly,face", [(0.3, -1), (2.0, -1), (0.5, 3), (1.7, 3)])
def test_rect_mc_transport_matches_oracle(orc, Ly, face):
    binding = require_gpu()
    from paper_2512_13965_amd import transport
    prob = _rect_problem(Ly, face, 60)
    n = 20_000
    w = binding.World(1 << 17, 1, 1 << 12)
    g = transport.run_problem(w, prob, n, 17, binding.SAMPLER_MC)
    w.close()
    o = orc.transport(prob, seed=17, h_begin=0, h_end=n, nthreads=8)
    rel = np.abs(g["flux"] - o["flux"]).sum() / np.abs(o["flux"]).sum()
    print(f"Ly {Ly} face {face}: flux L1 {rel:.2e}, leak {g['leak'].sum():.4f} vs {o['leak']:.4f}")
    assert rel < 5e-5
    assert abs(g["absorbed"].sum() + g["leak"].sum() + g["cutoff"].sum() - n) < 1e-9 * n


def test_rect_gmc_transport_runs_and_balances():
    # an 11-input model (random weights) steps a rectangular grid; square grids still run it
    binding = require_gpu()
    from paper_2512_13965_amd import transport
    m = binding.Model(inputs.pack_blob(inputs.random_weights(256, 3, n_in=11)), "bf16")
    w = binding.World(1 << 16, 1, 1 << 12)
    for Ly in (0.4, 0.0):
        r = transport.run_problem(w, _rect_problem(Ly, -1, 61), 10_000, 5, binding.SAMPLER_GMC, m, 8)
        assert abs(r["absorbed"].sum() + r["leak"].sum() + r["cutoff"].sum() - 10_000) < 1e-6
    w.close()
    m.close()
