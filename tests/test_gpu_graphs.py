"""Captured transport steps (gmc_world_set_graphs; the serving row's launch graphs per
batch-size bucket): a world that replays HIP graphs must produce what direct launches produce.

The kernels are the same; only the FP64 tally atomics may add in another order, so tallies
agree to 1e-12 relative and step / transmission counts exactly.  Graphs are replayed many times
(one per step, the same graph for every step whose particle count falls in its bucket), with
the program's own eager launches and synchronisations between the replays.
"""
import numpy as np
import pytest
import torch

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _run(binding, prob, n, seed, sampler, model, K, graphs, chunk, integrator="euler", between=None):
    from paper_2512_13965_amd import transport
    w = binding.World(1 << 16, 2, max(prob.n_cells, 1 << 12))
    if graphs:
        w.set_graphs(True)
    if between is None:
        out = transport.run_problem(w, prob, n, seed, sampler, model, K, chunk=chunk, integrator=integrator)
    else:
        # drive the steps by hand and launch unrelated eager work between replays
        w.set_integrator(integrator)
        pid = w.add_problem(prob, seed)
        injected, alive, steps = 0, 0, 0
        while injected < n or alive > 0:
            if injected < n and w.capacity - alive >= min(chunk, n - injected):
                cnt = min(chunk, n - injected)
                alive = w.inject(pid, injected, cnt)
                injected += cnt
            if alive > 0:
                alive = w.step(sampler, model, K)
                steps += 1
                between()
        out = w.tally(pid)
        w.remove(pid)
        out["steps"] = steps
    w.close()
    return out


def _same(a, b, n):
    for k in ("flux", "absorbed", "leak", "cutoff"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-12 * n)


@pytest.mark.parametrize("sampler", ["mc", "gmc", "gmc_split", "gmc_film"])
def test_graph_steps_match_direct_launches(sampler):
    binding = require_gpu()
    prob = inputs.checkerboard_problem(16, src=2)
    n = 30_000
    model = None
    if sampler == "gmc_film":
        # the residual network with adaptive modulation (its own kernel, eight waves)
        model = binding.Model(inputs.pack_blob(inputs.random_film_weights(256, 3)), "bf16")
    elif sampler != "mc":
        # gmc_split: a model flagged as fitted on collided crossings (first-flight split step)
        flags = 2 if sampler == "gmc_split" else 0
        model = binding.Model(inputs.pack_blob(inputs.random_weights(256, 3, flags=flags)), "bf16")
    smp = binding.SAMPLER_MC if sampler == "mc" else binding.SAMPLER_GMC
    # chunks of 7,000 give particle counts in several buckets (1024 .. 16384)
    eager = _run(binding, prob, n, 5, smp, model, 16, False, 7_000)
    graph = _run(binding, prob, n, 5, smp, model, 16, True, 7_000)
    assert graph["steps"] == eager["steps"] and graph["transmissions"] == eager["transmissions"]
    _same(graph, eager, n)
    if model is not None:
        model.close()


def test_graph_steps_of_a_grid_with_several_workgroups_per_cu():
    # width 128: the four-wave kernel's persistent grid holds several workgroups per CU once a
    # step has more than 128 samples per CU (chunks of 60,000 particles); the grid size, taken
    # from the occupancy query when the model is created, is baked into each captured graph
    binding = require_gpu()
    prob = inputs.checkerboard_problem(16, src=2)
    n = 120_000
    model = binding.Model(inputs.pack_blob(inputs.random_weights(128, 3)), "bf16")
    eager = _run(binding, prob, n, 8, binding.SAMPLER_GMC, model, 4, False, 60_000)
    graph = _run(binding, prob, n, 8, binding.SAMPLER_GMC, model, 4, True, 60_000)
    model.close()
    assert graph["steps"] == eager["steps"] and graph["transmissions"] == eager["transmissions"]
    _same(graph, eager, n)


def test_graph_replays_with_eager_work_between():
    binding = require_gpu()
    prob = inputs.checkerboard_problem(8, src=2)
    n = 20_000
    model = binding.Model(inputs.pack_blob(inputs.random_weights(256, 4)), "fp32")
    cond = binding.DeviceCond.from_host(inputs.transmission_conditions(5000, 9))
    scratch = torch.zeros(1 << 20, device="cuda")

    def between():
        binding.gmc_transmit(model, cond, 4, 1, 0)      # other kernels on the same stream
        scratch.add_(1.0)
        torch.cuda.synchronize()

    eager = _run(binding, prob, n, 11, binding.SAMPLER_GMC, model, 8, False, 4_000, between=between)
    graph = _run(binding, prob, n, 11, binding.SAMPLER_GMC, model, 8, True, 4_000, between=between)
    assert graph["steps"] == eager["steps"] and graph["steps"] > 10
    _same(graph, eager, n)
    model.close()


def test_graph_steps_follow_the_integrator_and_model():
    # a captured step is keyed by the integrator and the model: switching either re-captures
    binding = require_gpu()
    prob = inputs.checkerboard_problem(8, src=2)
    n = 8_000
    m1 = binding.Model(inputs.pack_blob(inputs.random_weights(256, 5)), "bf16")
    m2 = binding.Model(inputs.pack_blob(inputs.random_weights(256, 6)), "bf16")
    from paper_2512_13965_amd import transport
    w = binding.World(1 << 15, 2, 1 << 12)
    w.set_graphs(True)
    res = {}
    for name, m, integ in (("m1e", m1, "euler"), ("m2e", m2, "euler"), ("m1r", m1, "rk4"), ("m1e2", m1, "euler")):
        res[name] = transport.run_problem(w, prob, n, 3, binding.SAMPLER_GMC, m, 8, integrator=integ)
    w.close()
    ref = {}
    for name, m, integ in (("m1e", m1, "euler"), ("m2e", m2, "euler"), ("m1r", m1, "rk4")):
        w = binding.World(1 << 15, 2, 1 << 12)
        ref[name] = transport.run_problem(w, prob, n, 3, binding.SAMPLER_GMC, m, 8, integrator=integ)
        w.close()
    for name in ("m1e", "m2e", "m1r"):
        _same(res[name], ref[name], n)
    _same(res["m1e2"], ref["m1e"], n)
    assert not np.allclose(res["m1e"]["flux"], res["m2e"]["flux"])
    m1.close()
    m2.close()
