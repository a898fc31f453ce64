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
