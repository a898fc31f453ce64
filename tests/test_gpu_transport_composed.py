"""GMC-mode transport on the GPU against the oracle's transport composition (paper "Transport
Algorithm", stages 1-4 with the generative sampler as stage 2: the velocity network of eq. 8,
the decoder of eq. 11).

Both sides draw the same random numbers for every cell visit (noise of stream h + 2^32 visit),
so a history takes the same cells on both unless a decision falls the other way between FP32
on the GPU and FP64 in the oracle: a decoded face whose a4 lies within 1e-4 of a threshold, a
first-flight split within 1e-4 of its probability, a weight within 1e-5 of the cutoff.  The
oracle lists those histories (`at_risk`); their rate is reported and bounded, and the GPU and
the oracle then run the other histories, whose tallies must agree cell by cell."""
import numpy as np
import pytest

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu
from tests.test_gpu_transport import per_cell_ok

pytestmark = pytest.mark.gpu


def gpu_histories(binding, world, prob, seed, hist, model, K, integrator):
    """Runs exactly the histories `hist` of `prob` on the GPU (contiguous runs injected as bank
    slots free up) with the generative sampler; returns the per-cell tallies."""
    world.set_integrator(integrator)
    world.set_source_model(None, 16)
    pid = world.add_problem(prob, seed)
    hist = np.unique(np.asarray(hist, np.int64))
    runs = np.split(hist, np.nonzero(np.diff(hist) != 1)[0] + 1)
    alive = 0
    for r in runs:
        h0, left = int(r[0]), int(r.size)
        while left:
            free = world.capacity - alive
            if free <= 0:
                alive = world.step(binding.SAMPLER_GMC, model, K)
                continue
            cnt = min(left, free)
            alive = world.inject(pid, h0, cnt)
            h0 += cnt
            left -= cnt
    while alive:
        alive = world.step(binding.SAMPLER_GMC, model, K)
    t = world.tally(pid)
    world.remove(pid)
    return t


_T = np.tile(np.array([0.3, 2.0, 0.7, 1.5, 0.5, 3.0, 0.9, 0.2]), 8)
_C = np.tile(np.array([0.9, 0.5, 0.99, 0.7, 0.8, 0.95, 0.3, 0.6]), 8)

CASES = [
    # name, problem, model inputs, blob flags, integrator, K
    ("square_euler", inputs.Problem(8, 8, 0.5, _T, _C, 3, 3, 2, 2), 10, 0, "euler", 8),
    ("square_rk4", inputs.Problem(8, 8, 0.5, _T, _C, 3, 3, 2, 2), 10, 0, "rk4", 3),
    ("rect_surface_euler", inputs.Problem(8, 8, 0.5, _T, _C, 0, 0, 1, 8, src_face=3, Ly=0.3), 11, 0, "euler", 8),
    ("rect_tall_rk4", inputs.Problem(8, 8, 0.5, _T, _C, 3, 3, 2, 2, Ly=0.9), 11, 0, "rk4", 2),
    ("split_square_euler", inputs.Problem(8, 8, 0.5, _T, _C, 3, 3, 2, 2), 10, 2, "euler", 8),
    ("split_rect_rk4", inputs.Problem(8, 8, 0.5, _T, _C, 3, 3, 2, 2, Ly=0.7), 11, 2, "rk4", 2),
]


@pytest.mark.parametrize("name,prob,n_in,flags,integ,K", CASES, ids=[c[0] for c in CASES])
def test_gmc_transport_matches_oracle_composition(orc, name, prob, n_in, flags, integ, K):
    binding = require_gpu()
    n, seed = 1500, 31
    w = inputs.random_weights(128, 40 + n_in + flags, n_in=n_in, flags=flags)
    stage2 = orc.stage2_generative(w, K, integ)
    full = orc.transport_composed(prob, seed, np.arange(n), stage2)
    risk = np.array(full["at_risk"], np.int64)
    safe = np.setdiff1d(np.arange(n), risk)
    ref = orc.transport_composed(prob, seed, safe, stage2) if risk.size else full
    frac = risk.size / n
    print(f"{name}: {full['events']:.0f} transmissions, {risk.size} histories at risk ({frac:.2%}), "
          f"{full['rejected_n'].sum():.0f} rejected samples")
    assert frac < 0.05
    m = binding.Model(inputs.pack_blob(w), "fp32")
    world = binding.World(1 << 12, 1, 1 << 8)
    world.set_streaming(64 if flags & 2 else 1)
    g = gpu_histories(binding, world, prob, seed, safe, m, K, integ)
    world.close()
    m.close()
    ns = safe.size
    for k in ("flux", "absorbed", "leak", "cutoff", "wpath", "path", "visits"):
        ok, worst = per_cell_ok(g[k], ref[k], ns)
        print(f"{name}: {k} per-cell worst ratio to the bound {worst:.2e}")
        assert ok, (k, worst)
    assert g["rejected_n"].sum() == ref["rejected_n"].sum()
    bal = g["leak"].sum() + g["absorbed"].sum() + g["cutoff"].sum()
    assert abs(bal - ns) < 1e-9 * ns


FILM_CASES = [
    ("film_square_euler", inputs.Problem(8, 8, 0.5, _T, _C, 3, 3, 2, 2), 10, 0, "euler", 8),
    ("film_rect_rk4", inputs.Problem(8, 8, 0.5, _T, _C, 3, 3, 2, 2, Ly=0.7), 11, 0, "rk4", 2),
    ("film_split_square_euler", inputs.Problem(8, 8, 0.5, _T, _C, 3, 3, 2, 2), 10, 2, "euler", 8),
]


@pytest.mark.parametrize("name,prob,n_in,flags,integ,K", FILM_CASES, ids=[c[0] for c in FILM_CASES])
def test_gmc_transport_with_the_residual_network(orc, name, prob, n_in, flags, integ, K):
    # the same composition with the residual velocity network with adaptive modulation as the
    # stage-2 sampler (FP32, H = 128, random-init)
    binding = require_gpu()
    n, seed = 1200, 37
    w = inputs.random_film_weights(128, 60 + n_in + flags, n_in=n_in, flags=flags)
    stage2 = orc.stage2_generative(w, K, integ)
    full = orc.transport_composed(prob, seed, np.arange(n), stage2)
    risk = np.array(full["at_risk"], np.int64)
    safe = np.setdiff1d(np.arange(n), risk)
    ref = orc.transport_composed(prob, seed, safe, stage2) if risk.size else full
    print(f"{name}: {full['events']:.0f} transmissions, {risk.size} histories at risk ({risk.size / n:.2%})")
    assert risk.size / n < 0.05
    m = binding.Model(inputs.pack_blob(w), "fp32")
    world = binding.World(1 << 12, 1, 1 << 8)
    world.set_streaming(64 if flags & 2 else 1)
    g = gpu_histories(binding, world, prob, seed, safe, m, K, integ)
    world.close()
    m.close()
    for k in ("flux", "absorbed", "leak", "cutoff", "wpath", "path", "visits"):
        ok, worst = per_cell_ok(g[k], ref[k], safe.size)
        print(f"{name}: {k} per-cell worst ratio to the bound {worst:.2e}")
        assert ok, (k, worst)
    assert g["rejected_n"].sum() == ref["rejected_n"].sum()
