"""Continuous batching on the GPU: a request's result is the same served alone and served in a
stream of other requests that share its transport steps (same seed -> same random numbers)."""
import numpy as np
import pytest

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("sampler", ["gmc", "mc"])
def test_request_alone_and_in_mix(sampler):
    binding = require_gpu()
    from paper_2512_13965_amd import serving
    model = None
    smp = binding.SAMPLER_MC
    if sampler == "gmc":
        model = binding.Model(inputs.pack_blob(inputs.random_weights(256, 3)), "bf16")
        smp = binding.SAMPLER_GMC
    world = binding.World(1 << 17, 8, 1 << 16)
    prob = inputs.checkerboard_problem(8, src=2)
    target = serving.Request(0, prob, 20_000, seed=77, arrival=0.0)
    alone = serving.Server(world, smp, model, K=8).run([target])
    others = serving.poisson_requests(
        6, rate_hz=200.0, seed=5,
        make_problem=lambda i: inputs.random_problem(100 + i, side_range=(16, 32),
                                                     hist_log10_range=(4.0, 4.5)))
    again = serving.Request(100, prob, 20_000, seed=77, arrival=0.005)
    mix = serving.Server(world, smp, model, K=8).run(others + [again])
    world.close()
    assert len(mix.requests) == 7
    for k in ("flux", "absorbed", "leak", "cutoff"):
        np.testing.assert_allclose(again.tallies[k], target.tallies[k], rtol=1e-12,
                                   atol=1e-12 * target.n_hist)
    for r in mix.requests:
        tot = sum(r.tallies[k].sum() for k in ("absorbed", "leak", "cutoff"))
        assert abs(tot - r.n_hist) < 1e-9 * r.n_hist          # every history accounted for
        assert r.latency > 0
    p = mix.latency_percentiles()
    assert p["p99"] >= p["p50"] > 0
    assert mix.transmissions > 0 and mix.steps > 0


def test_served_requests_match_the_oracle(orc):
    # every request of a Poisson stream served with the analog sampler against the oracle's
    # transport of the same problem and seed (the same random numbers per history and cell
    # visit): per cell |d| <= 1e-4 |phi| + 1e-9 N, leak and absorption within 1e-3 per history
    binding = require_gpu()
    from paper_2512_13965_amd import serving
    from tests.test_gpu_transport import check_within_noise, oracle_batches, per_cell_ok
    world = binding.World(1 << 17, 8, 1 << 16)
    reqs = serving.poisson_requests(
        8, rate_hz=300.0, seed=9,
        make_problem=lambda i: inputs.random_problem(300 + i, side_range=(16, 40), hist_log10_range=(3.5, 4.3)))
    st = serving.Server(world, binding.SAMPLER_MC, None).run(reqs)
    world.close()
    assert len(st.requests) == len(reqs)
    for r in st.requests:
        o, se = oracle_batches(orc, r.problem, r.seed, r.n_hist)
        n = r.n_hist
        for k in ("flux", "absorbed"):
            ok, worst = per_cell_ok(r.tallies[k], o[k], n)
            print(f"request {r.rid} ({r.problem.nx}^2, {n} histories): {k} worst ratio {worst:.2e}")
            assert ok, (r.rid, k, worst)
        check_within_noise(r.tallies, o, se, n, f"request {r.rid}")
        assert abs(r.tallies["leak"].sum() - o["leak"]) <= 1e-3 * n
        assert abs(r.tallies["absorbed"].sum() - o["absorbed"].sum()) <= 1e-3 * n


def test_served_generative_requests_match_the_oracle_composition(orc):
    # requests served with the generative sampler (FP32, H = 128, random-init, Euler K = 4)
    # against the oracle's transport composition with the same network; each request's seed is
    # the first for which the oracle lists no history at risk of an FP32 / FP64 decision flip
    binding = require_gpu()
    from paper_2512_13965_amd import serving
    from tests.test_gpu_transport import per_cell_ok
    w = inputs.random_weights(128, 61)
    stage2 = orc.stage2_generative(w, 4)
    reqs, refs = [], []
    for i in range(4):
        prob, _ = inputs.random_problem(500 + i, side_range=(8, 12))
        n = 400 + 100 * i
        for seed in range(1000 * (i + 1), 1000 * (i + 1) + 50):
            ref = orc.transport_composed(prob, seed, np.arange(n), stage2)
            if not ref["at_risk"]:
                break
        else:
            pytest.fail("no seed without histories at risk")
        reqs.append(serving.Request(i, prob, n, seed=seed, arrival=0.002 * i))
        refs.append(ref)
    m = binding.Model(inputs.pack_blob(w), "fp32")
    world = binding.World(1 << 14, 4, 1 << 12)
    st = serving.Server(world, binding.SAMPLER_GMC, m, K=4).run(reqs)
    world.close()
    m.close()
    assert len(st.requests) == len(reqs)
    for r in st.requests:
        ref = refs[r.rid]
        for k in ("flux", "absorbed", "leak", "cutoff", "wpath", "path", "visits"):
            ok, worst = per_cell_ok(r.tallies[k], ref[k], r.n_hist)
            print(f"generative request {r.rid}: {k} worst ratio {worst:.2e}")
            assert ok, (r.rid, k, worst)
