"""GPU transport (paper section "Transport Algorithm"; track-length tallies of eqs. 5-7)
against the FP64 oracle transport, the conservation laws and the statistical behaviour of
eq. 12.

With the analog sampler both sides draw the same Philox words for every history, so a history
takes the same path on both sides unless an FP32 near-tie sends the GPU walk the other way (see
test_gpu_walk.py); flux maps then agree far inside their statistical error.
"""
import math

import numpy as np
import pytest
import torch

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def per_cell_ok(g, o, n, rel=1e-4, abs_per_hist=1e-9):
    """Per-cell bound |g - o| <= rel * |o| + abs_per_hist * n; returns (ok, worst ratio)."""
    g, o = np.asarray(g, np.float64), np.asarray(o, np.float64)
    ratio = np.abs(g - o) / (rel * np.abs(o) + abs_per_hist * n)
    return bool(np.all(ratio <= 1.0)), float(ratio.max())


TALLIES = ("flux", "absorbed", "wpath", "path", "visits")


def oracle_batches(orc, prob, seed, n, batches=16):
    """The oracle's transport of histories [0, n) run in `batches` contiguous batches: their
    sums (the one-run result: histories are independent of the chunking) and the standard error
    of each per-cell sum, sqrt(batches) times the spread of the batch sums."""
    parts = [orc.transport(prob, seed=seed, h_begin=n * b // batches, h_end=n * (b + 1) // batches, nthreads=8)
             for b in range(batches)]
    ref = {k: np.sum([p[k] for p in parts], axis=0) for k in TALLIES}
    ref["leak"] = sum(p["leak"] for p in parts)
    se = {k: np.std([p[k] for p in parts], axis=0, ddof=1) * math.sqrt(batches) for k in TALLIES}
    return ref, se


def check_within_noise(g, ref, se, n, label):
    """Analog transport, GPU against the oracle on the same random numbers, per cell: the
    difference must stay below 1e-4 |ref| + 1e-9 n plus half the cell's own statistical
    standard error (measured: at most a tenth of it).  A history takes the same cells on both sides unless an FP32 near-tie sends the GPU
    walk the other way (a few in 10^7 flights, see test_gpu_walk.py); such a history moves the
    tallies of the cells it touches by less than their noise, while a wrong tally in a low-flux
    cell (hidden in a map-wide L1 norm) would not be."""
    for k in TALLIES:
        d = np.abs(np.asarray(g[k], np.float64) - ref[k])
        ratio = d / (1e-4 * np.abs(ref[k]) + 1e-9 * n + 0.5 * se[k])
        strict = d / (1e-4 * np.abs(ref[k]) + 1e-9 * n)
        print(f"{label}: {k} worst ratio to the bound {ratio.max():.2e} (to 1e-4 |ref| + 1e-9 n alone: "
              f"{strict.max():.2e}, cells over it {int((strict > 1).sum())})")
        assert ratio.max() <= 1.0, (k, ratio.max())


def _gpu(binding, prob, n, seed, sampler, model=None, K=16, capacity=1 << 18):
    from paper_2512_13965_amd import transport
    w = binding.World(capacity, 2, max(prob.n_cells, 1 << 12))
    out = transport.run_problem(w, prob, n, seed, sampler, model, K)
    w.close()
    return out


@pytest.mark.parametrize("name,prob", [
    ("checkerboard8", inputs.checkerboard_problem(8, src=2)),
    ("hetero3", inputs.Problem(3, 3, 0.7, np.array([0.3, 2.0, 0.7, 1.5, 0.5, 3.0, 0.9, 0.2, 1.1]),
                               np.array([0.9, 0.5, 0.99, 0.7, 0.8, 0.95, 0.3, 1.0, 0.6]), 1, 1, 1, 1)),
])
def test_mc_transport_matches_oracle(orc, name, prob):
    binding = require_gpu()
    n = 20_000
    g = _gpu(binding, prob, n, seed=11, sampler=binding.SAMPLER_MC)
    o, se = oracle_batches(orc, prob, 11, n)
    rel = np.abs(g["flux"] - o["flux"]).sum() / np.abs(o["flux"]).sum()
    print(f"{name}: flux L1 rel diff {rel:.2e}; leak {g['leak'].sum():.6f} vs {o['leak']:.6f}; "
          f"absorbed {g['absorbed'].sum():.6f} vs {o['absorbed'].sum():.6f}")
    assert rel < 5e-5          # measured <= 3e-6
    assert abs(g["leak"].sum() - o["leak"]) <= 1e-3 * n
    assert abs(g["absorbed"].sum() - o["absorbed"].sum()) <= 1e-3 * n
    # per cell: a low-flux cell must not hide inside the map's total
    check_within_noise(g, o, se, n, name)
    # every visit is a birth leg or a transmission of a step
    assert g["visits"].sum() == n + g["transmissions"]


@pytest.mark.parametrize("sampler", ["mc", "gmc"])
def test_weight_balance(sampler):
    # every unit of source weight leaks, is absorbed or is cut off -- for any sampler, since
    # the tally is the weight lost along the sampled path
    binding = require_gpu()
    prob = inputs.checkerboard_problem(16, src=2)
    n = 50_000
    model = None
    if sampler == "gmc":
        model = binding.Model(inputs.pack_blob(inputs.random_weights(256, 1)), "bf16")
    g = _gpu(binding, prob, n, 3, binding.SAMPLER_MC if sampler == "mc" else binding.SAMPLER_GMC, model)
    total = g["leak"].sum() + g["absorbed"].sum() + g["cutoff"].sum()
    assert abs(total - n) < 1e-9 * n
    assert np.all(g["flux"] >= 0) and g["transmissions"] >= n


def test_reflecting_box_flux_equals_source_over_sigma_a():
    # P7: reflecting homogeneous box with a uniform source: E[phi_i] = N / (sigma_a V n_cells)
    binding = require_gpu()
    tau, c, L = 2.0, 0.8, 0.5
    prob = inputs.homogeneous_problem(6, tau, c, reflect=True, L=L)
    n = 200_000
    g = _gpu(binding, prob, n, 5, binding.SAMPLER_MC)
    sig_a, V = (1 - c) * tau / L, L * L
    assert g["leak"].sum() == 0.0
    assert abs(g["absorbed"].sum() + g["cutoff"].sum() - n) < 1e-9 * n
    np.testing.assert_allclose((g["flux"] * sig_a * V).sum(), g["absorbed"].sum(), rtol=1e-12)
    phi = n / (sig_a * V * prob.n_cells)
    assert abs(g["flux"].mean() - phi) / phi < 2e-3
    assert np.abs(g["flux"] / phi - 1).max() < 0.05


@pytest.mark.parametrize("sampler", ["mc", "gmc"])
def test_alone_and_in_mix_agree(sampler):
    # a problem's tallies do not depend on the other problems sharing the bank
    binding = require_gpu()
    from paper_2512_13965_amd import transport
    a = inputs.checkerboard_problem(8, src=2)
    b, _ = inputs.random_problem(7, side_range=(16, 24))
    model = None
    if sampler == "gmc":
        model = binding.Model(inputs.pack_blob(inputs.random_weights(256, 2)), "fp32")
    smp = binding.SAMPLER_MC if sampler == "mc" else binding.SAMPLER_GMC
    na, nb = 20_000, 30_000
    w = binding.World(1 << 17, 4, 1 << 12)
    alone = transport.run_problem(w, a, na, 21, smp, model)
    # the mix: b first (other slot and cells), then a, injected and stepped together
    pb = w.add_problem(b, 99)
    pa = w.add_problem(a, 21)
    w.inject(pb, 0, nb)
    w.inject(pa, 0, na)
    alive = 1
    while alive:
        alive = w.step(smp, model)
    mix = w.tally(pa)
    w.close()
    for k in ("flux", "absorbed", "leak", "cutoff"):
        np.testing.assert_allclose(mix[k], alone[k], rtol=1e-12, atol=1e-12 * na)


def test_cfg3_checkerboard_gpu_vs_oracle(orc):
    # 32 x 32 unit cells, checkerboard (0.5, 0.5) / (50, 0.99), central 4 x 4 source, vacuum
    binding = require_gpu()
    prob = inputs.checkerboard_problem(32)
    n = 100_000
    g = _gpu(binding, prob, n, 1, binding.SAMPLER_MC, capacity=1 << 20)
    o, se = oracle_batches(orc, prob, 1, n)
    rel = np.abs(g["flux"] - o["flux"]).sum() / np.abs(o["flux"]).sum()
    print(f"cfg3: flux L1 rel diff {rel:.2e}, transmissions {g['transmissions']}, steps {g['steps']}")
    assert rel < 5e-5          # measured <= 3e-6
    assert abs(g["absorbed"].sum() + g["leak"].sum() + g["cutoff"].sum() - n) < 1e-9 * n
    check_within_noise(g, o, se, n, "cfg3")


def test_eq12_error_decays_as_inverse_sqrt_n():
    # eq. 12: cell-averaged standard deviation over K = 5 independent runs, log-log slope -1/2
    binding = require_gpu()
    prob = inputs.checkerboard_problem(16, src=2)
    Ns = [10_000, 40_000, 160_000]
    sig = []
    for N in Ns:
        runs = np.array([_gpu(binding, prob, N, 1000 + 17 * k, binding.SAMPLER_MC)["flux"] / N
                         for k in range(5)])
        sig.append(np.mean(runs.std(0, ddof=1)))
    slope = np.polyfit(np.log(Ns), np.log(sig), 1)[0]
    print("eq12 sigma", sig, "slope", slope)
    assert abs(slope + 0.5) < 0.1


def test_eq12_generative_transport_converges_like_mc():
    # eq. 12 with the generative sampler ("Convergence and Performance": the GMC and MC curves of
    # sigma(N) coincide): the fitted H = 128 collided model with the first-flight split on the
    # paper's lattice decays as N^-1/2 with the analog runs' spread
    binding = require_gpu()
    import os
    from paper_2512_13965_amd import transport
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2512_13965_amd",
                        "weights", "gmc_h128_collided.bin")
    if not os.path.exists(path):
        pytest.skip("no fitted weights")
    m = binding.Model(open(path, "rb").read(), "bf16")
    prob = inputs.lattice_problem(16)
    w = binding.World(1 << 18, 1, 1 << 14)
    Ns = [20_000, 80_000, 320_000]
    sig = {}
    for kind, smp, mm in (("mc", binding.SAMPLER_MC, None), ("gmc", binding.SAMPLER_GMC, m)):
        s = []
        for N in Ns:
            runs = np.array([transport.run_problem(w, prob, N, 3000 + 13 * k, smp, mm, 12, integrator="rk4")["flux"] / N
                             for k in range(5)])
            s.append(np.mean(runs.std(0, ddof=1)))
        sig[kind] = np.array(s)
    w.close()
    m.close()
    slopes = {k: np.polyfit(np.log(Ns), np.log(v), 1)[0] for k, v in sig.items()}
    print("eq12 lattice sigma", sig, "slopes", slopes)
    assert abs(slopes["gmc"] + 0.5) < 0.1 and abs(slopes["mc"] + 0.5) < 0.1
    assert np.all(np.abs(sig["gmc"] / sig["mc"] - 1) < 0.1)


def test_world_errors():
    binding = require_gpu()
    w = binding.World(1000, 1, 100)
    with pytest.raises(binding.GmcError):
        w.add_problem(inputs.checkerboard_problem(16), 1)          # 256 cells > 100
    pid = w.add_problem(inputs.checkerboard_problem(8, src=2), 1)
    with pytest.raises(binding.GmcError):
        w.add_problem(inputs.checkerboard_problem(4, src=2), 2)     # no free slot
    with pytest.raises(binding.GmcError):
        w.inject(pid, 0, 2000)                                       # more than the bank holds
    n = w.inject(pid, 0, 500)
    assert 0 <= n <= 500
    if n:
        with pytest.raises(binding.GmcError):
            w.remove(pid)                                            # still in flight
    while n:
        n = w.step(binding.SAMPLER_MC)
    w.remove(pid)
    w.close()


def test_visit_cap_matches_oracle_and_ends_every_history(orc):
    # a reflecting box without absorption: every history runs into the visit cap (visits
    # 0 .. M-1, the birth leg in inject and M - 1 transmissions in steps) and is cut off
    binding = require_gpu()
    from paper_2512_13965_amd import transport
    n, M = 20_000, 50
    prob = inputs.homogeneous_problem(4, 1.0, 1.0, reflect=True)
    prob.max_visits = M
    w = binding.World(1 << 15, 1, 1 << 8)
    g = transport.run_problem(w, prob, n, 3, binding.SAMPLER_MC)
    o = orc.transport(prob, seed=3, h_begin=0, h_end=n, nthreads=8)
    rel = np.abs(g["flux"] - o["flux"]).sum() / np.abs(o["flux"]).sum()
    print(f"visit cap: flux L1 rel diff {rel:.2e}, steps {g['steps']}")
    assert rel < 5e-5
    assert g["cutoff"].sum() == pytest.approx(n, rel=1e-12) and g["leak"].sum() == 0.0
    assert g["transmissions"] == (M - 1) * n
    # the same cap inside the split's streamed crossings: a thin non-scattering medium, so every
    # crossing is uncollided and the split step equals the walk step
    prob2 = inputs.homogeneous_problem(4, 1e-3, 0.0, reflect=True)
    prob2.max_visits = M
    m = binding.Model(inputs.pack_blob(inputs.random_weights(128, 5, flags=2)), "fp32")
    g1 = transport.run_problem(w, prob2, n, 4, binding.SAMPLER_MC)
    g2 = transport.run_problem(w, prob2, n, 4, binding.SAMPLER_GMC, m, 4)
    w.close()
    m.close()
    for r in (g1, g2):
        # the thin absorber takes a few per cent; the cap takes the rest, nothing leaks
        assert r["cutoff"].sum() + r["absorbed"].sum() == pytest.approx(n, rel=1e-9)
        assert r["leak"].sum() == 0.0 and r["cutoff"].sum() > 0.9 * n
        assert r["transmissions"] == (M - 1) * n
    assert g2["cutoff"].sum() == pytest.approx(g1["cutoff"].sum(), rel=1e-6)
    assert np.abs(g2["flux"] - g1["flux"]).sum() / np.abs(g1["flux"]).sum() < 1e-6
    assert g2["steps"] < g1["steps"]


def test_p3_mean_track_per_cell_visit_on_gpu(orc):
    # P3 per cell type on the GPU path tallies: reflecting 4 x 4 checkerboard of pure scatterers
    # (tau = 0.5 / 20), histories cut at visit M; the difference between two caps holds the
    # visits M1 .. M2 - 1, whose mean track is pi L / 4 in every cell type (mean-chord
    # invariance); and the GPU's differences equal the oracle's per cell
    binding = require_gpu()
    from paper_2512_13965_amd import transport
    t = np.where((np.arange(4)[:, None] + np.arange(4)[None, :]) % 2 == 0, 0.5, 20.0).reshape(-1)
    L, n = 0.5, 50_000
    prob = inputs.Problem(4, 4, L, t, np.ones(16), 0, 0, 4, 4, reflect=True)
    w = binding.World(1 << 17, 1, 1 << 8)
    g, o = {}, {}
    for M in (16, 64):
        prob.max_visits = M
        g[M] = transport.run_problem(w, prob, n, 8, binding.SAMPLER_MC)
        o[M] = oracle_batches(orc, prob, 8, n)
    w.close()
    dl, dv = g[64]["path"] - g[16]["path"], g[64]["visits"] - g[16]["visits"]
    assert dv.sum() == 48 * n
    for sel in (t == 0.5, t == 20.0):
        mean = dl[sel].sum() / dv[sel].sum()
        tol = 4 * L * math.sqrt(4.0 / dv[sel].sum())
        print(f"P3 cell type tau={t[sel][0]:g}: mean track per visit {mean:.5f} vs pi L / 4 = {math.pi * L / 4:.5f}")
        assert abs(mean - math.pi * L / 4) < tol
    for M in (16, 64):
        check_within_noise(g[M], o[M][0], o[M][1], n, f"cap {M}")
