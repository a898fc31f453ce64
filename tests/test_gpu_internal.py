"""GPU parity of the internal (volumetric-source) model path: the analog walk started inside
the cell (mc_transmit_internal) and the generative sampler with the 12-input network
(gmc_sample_internal) against the FP64 oracle, and transport births sampled by an internal
model (gmc_world_set_source_model).

Tolerances are those of the boundary-model tests (test_gpu_walk.py, test_gpu_sampler.py): the
kernels are the same; only the walk's start point and the network's input width differ.
"""
import numpy as np
import pytest
import torch

from paper_2512_13965_amd import inputs
from tests.gpu_util import face_threshold_margin, require_gpu, sample_indices

pytestmark = pytest.mark.gpu
NI = inputs.N_IN_INTERNAL


def _walk(binding, cond, mode, seed, id_base=0):
    dc = binding.DeviceCondInternal.from_host(cond)
    nc = torch.empty(len(cond), dtype=torch.int32, device="cuda")
    out = binding.mc_transmit_internal(dc, mode, seed, id_base, ncoll=nc)
    torch.cuda.synchronize()
    h = out.to_host()
    h["ncoll"] = nc.cpu().numpy().astype(np.int64)
    return h


def _compare(g, o, max_mismatch=5e-4):
    same = (g["face"] == o["face"]) & (g["ncoll"] == o["ncoll"].astype(np.int64))
    frac = 1.0 - same.mean()
    d_pos = np.abs(g["pos"][same] - o["pos"][same])
    d_dir = np.maximum(np.abs(g["dir_cos"][same] - o["u"][same]), np.abs(g["dir_sin"][same] - o["v"][same]))
    d_len = np.abs(g["path"][same] - o["len"][same]) / np.maximum(o["len"][same], 1e-6)
    print(f"mismatch {frac:.2e} pos {d_pos.max():.2e} dir {d_dir.max():.2e} len p99.9 {np.quantile(d_len, .999):.2e}")
    assert frac <= max_mismatch
    assert d_pos.max() < 1e-4 and d_dir.max() < 1e-5
    assert np.quantile(d_len, 0.999) < 1e-5 and d_len.max() < 1e-3


@pytest.mark.parametrize("tau", [1.0, 10.0, 100.0])
def test_internal_walk_matches_oracle(orc, tau):
    binding = require_gpu()
    cond = inputs.fixed_internal_conditions(1 << 16, tau, 1.0, seed=41)
    _compare(_walk(binding, cond, binding.MODE_CONTINUOUS, 3), orc.mc_transmit_internal(cond, 0, 3, nthreads=8))


def test_internal_walk_mixed_cells_and_analog_absorption(orc):
    binding = require_gpu()
    cond = inputs.internal_conditions(60_001, seed=42)
    _compare(_walk(binding, cond, binding.MODE_CONTINUOUS, 4, 999),
             orc.mc_transmit_internal(cond, 0, 4, 999, nthreads=8))
    cond = inputs.fixed_internal_conditions(20_000, 2.0, 0.7, seed=43)
    g = _walk(binding, cond, binding.MODE_ANALOG, 5)
    _compare(g, orc.mc_transmit_internal(cond, 1, 5, nthreads=8))
    assert np.any(g["face"] == -1)


def _sample(binding, w, prec, cond, integ, K, seed=2, noise=None):
    m = binding.Model(inputs.pack_blob(w), prec)
    assert m.n_in == NI
    dc = binding.DeviceCondInternal.from_host(cond)
    n = len(cond)
    raw = torch.empty(5 * n, dtype=torch.float32, device="cuda")
    nz = None if noise is None else torch.from_numpy(noise.reshape(-1)).cuda()
    out = binding.gmc_sample_internal(m, dc, integ, K, seed, 0, noise=nz, raw=raw)
    torch.cuda.synchronize()
    m.close()
    return raw.view(5, n).cpu().numpy().astype(np.float64), out.to_host()


def _z(orc, idx, seed):
    return np.stack([orc.noise(seed, int(i), 1)[:, 0] for i in idx], axis=1)


@pytest.mark.parametrize("integ,K", [("euler", 16), ("rk4", 6)])
def test_internal_sampler_fp32_parity(orc, integ, K):
    binding = require_gpu()
    n = 20_011
    cond = inputs.internal_conditions(n, seed=44)
    w = inputs.random_weights(256, 7, n_in=NI)
    raw, out = _sample(binding, w, "fp32", cond, integ, K)
    idx = sample_indices(n, 500)
    sampler = orc.sample_raw if integ == "euler" else orc.sample_raw_rk4
    ref = sampler(w, cond.subset(idx), K, _z(orc, idx, 2))
    err = np.abs(raw[:, idx].T - ref).max(axis=1)
    print(f"internal fp32 {integ}: max {err.max():.2e}")
    assert err.max() < 1e-5
    d = orc.decode(ref)
    far = face_threshold_margin(ref[:, 4]) > 1e-3
    np.testing.assert_array_equal(out["face"][idx][far], d["face"][far])


@pytest.mark.parametrize("prec,H", [("bf16", 512), ("fp8", 512), ("bf16", 256)])
def test_internal_sampler_quantised_parity(orc, prec, H):
    binding = require_gpu()
    n = 20_077
    cond = inputs.internal_conditions(n, seed=45)
    w = inputs.random_weights(H, 8, n_in=NI)
    z = inputs.noise(n, 9)
    raw, _ = _sample(binding, w, prec, cond, "euler", 16, noise=z)
    idx = sample_indices(n, 250, seed=3)
    oprec = orc.PREC_BF16_EXP2 if prec == "bf16" else orc.PREC_FP8_EXP2
    ref = orc.sample_raw(w, cond.subset(idx), 16, z[:, idx].astype(np.float64), oprec)
    exact = orc.sample_raw(w, cond.subset(idx), 16, z[:, idx].astype(np.float64), orc.PREC_FP64)
    err = np.abs(raw[:, idx].T - ref).max(axis=1)
    err_exact = np.abs(raw[:, idx].T - exact).max(axis=1)
    print(f"internal {prec} H={H}: p99 {np.quantile(err, .99):.2e} max {err.max():.2e}")
    if prec == "bf16":
        assert np.quantile(err, 0.99) < 1e-5 and err.max() < 5e-5
    else:
        assert np.quantile(err, 0.99) < 1e-4 and err.max() < 3e-4
    assert np.median(err) < 0.1 * np.median(err_exact)


def test_model_kind_is_checked():
    binding = require_gpu()
    mi = binding.Model(inputs.pack_blob(inputs.random_weights(128, 1, n_in=NI)), "fp32")
    mb = binding.Model(inputs.pack_blob(inputs.random_weights(128, 1)), "fp32")
    assert mi.n_in == 12 and mb.n_in == 10
    bc = binding.DeviceCond.from_host(inputs.transmission_conditions(10, 1))
    ic = binding.DeviceCondInternal.from_host(inputs.internal_conditions(10, 1))
    with pytest.raises(binding.GmcError):
        binding.gmc_sample(mi, bc, "euler", 4, 0)
    with pytest.raises(binding.GmcError):
        binding.gmc_sample_internal(mb, ic, "euler", 4, 0)
    w = binding.World(1 << 12, 1, 1 << 10)
    with pytest.raises(binding.GmcError):
        w.set_source_model(mb, 8)
    # an empty world: the check comes before any launch
    with pytest.raises(binding.GmcError):
        w.step(binding.SAMPLER_GMC, mi, 8)
    w.close()
    mi.close()
    mb.close()


def test_transport_with_internal_source_model():
    binding = require_gpu()
    from paper_2512_13965_amd import transport
    src = binding.Model(inputs.pack_blob(inputs.random_weights(256, 9, n_in=NI)), "bf16")
    bnd = binding.Model(inputs.pack_blob(inputs.random_weights(256, 10)), "bf16")
    a = inputs.checkerboard_problem(8, src=2)
    b, _ = inputs.random_problem(5, side_range=(16, 24))
    na, nb = 20_000, 15_000
    w = binding.World(1 << 16, 4, 1 << 12)
    alone = transport.run_problem(w, a, na, 21, binding.SAMPLER_GMC, bnd, 8, source_model=src, source_K=8)
    total = alone["leak"].sum() + alone["absorbed"].sum() + alone["cutoff"].sum()
    assert abs(total - na) < 1e-9 * na
    again = transport.run_problem(w, a, na, 21, binding.SAMPLER_GMC, bnd, 8, source_model=src, source_K=8)
    w.set_source_model(src, 8)
    pb = w.add_problem(b, 99)
    pa = w.add_problem(a, 21)
    w.inject(pb, 0, nb)
    w.inject(pa, 0, na)
    alive = 1
    while alive:
        alive = w.step(binding.SAMPLER_GMC, bnd, 8)
    mix = w.tally(pa)
    w.remove(pa)
    w.remove(pb)
    # without a source model the births take the analog first leg: other tallies
    analog_births = transport.run_problem(w, a, na, 21, binding.SAMPLER_GMC, bnd, 8)
    w.close()
    for k in ("flux", "absorbed", "leak", "cutoff"):
        np.testing.assert_allclose(again[k], alone[k], rtol=1e-12, atol=1e-12 * na)
        np.testing.assert_allclose(mix[k], alone[k], rtol=1e-12, atol=1e-12 * na)
    assert not np.array_equal(analog_births["flux"], alone["flux"])
    src.close()
    bnd.close()
