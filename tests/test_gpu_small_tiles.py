"""Sampler launches with at most 32 (64) samples per compute unit run 32-sample (64-sample)
tiles (the tail steps of a transport run, small requests).  Every accumulator sums its
k-blocks in the same order as with 128-sample tiles, so a sample's result does not depend on
the tile size: the samples of a small launch must equal, bit for bit, the same samples inside
a large launch (same conditions, same random-number ids), and match the rounding-emulating
oracle like any launch."""
import numpy as np
import pytest
import torch

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu
from tests.test_gpu_sampler import _oracle_raw

pytestmark = pytest.mark.gpu


def _raw(binding, m, cond_h, integ, K, n=None):
    dc = binding.DeviceCond.from_host(cond_h)
    n = len(cond_h) if n is None else n
    raw = torch.empty(5 * n, dtype=torch.float32, device="cuda")
    binding.gmc_sample(m, dc, integ, K, 7, 0, raw=raw, n=n)
    torch.cuda.synchronize()
    return raw.view(5, n).cpu().numpy()


def _small_limit():
    return 32 * torch.cuda.get_device_properties(0).multi_processor_count


@pytest.mark.parametrize("prec,H,integ,K", [("bf16", 512, "euler", 16), ("bf16", 256, "rk4", 3),
                                            ("fp8", 512, "euler", 8), ("fp8", 256, "rk4", 2)])
def test_small_launch_equals_the_same_samples_in_a_large_launch(prec, H, integ, K):
    binding = require_gpu()
    small = _small_limit()
    big = 8 * small                                   # 128-sample tiles
    cond = inputs.transmission_conditions(big, 21)
    m = binding.Model(inputs.pack_blob(inputs.random_weights(H, 22)), prec)
    ref = _raw(binding, m, cond, integ, K)
    for n in (1, 31, 32, 33, 1000, small, small + 1, 3 * small // 2, 2 * small, 2 * small + 1):
        got = _raw(binding, m, cond.subset(slice(0, n)), integ, K)
        np.testing.assert_array_equal(got, ref[:, :n], err_msg=f"n = {n}")
    m.close()


def _exits(binding, m, cond_h, integ, K, raw):
    dc = binding.DeviceCond.from_host(cond_h)
    n = len(cond_h)
    r = torch.empty(5 * n, dtype=torch.float32, device="cuda") if raw else None
    out = binding.gmc_sample(m, dc, integ, K, 7, 3, raw=r)
    torch.cuda.synchronize()
    return out.to_host()


@pytest.mark.parametrize("prec,H,integ,K", [("bf16", 512, "euler", 4), ("fp8", 256, "rk4", 1)])
def test_last_round_on_small_tiles_equals_one_launch(prec, H, integ, K):
    # a count known on the host whose last round of 128-sample tiles would hold at most 32 (64)
    # samples per compute unit runs that remainder as a second launch of 32-sample (64-sample)
    # tiles over the shifted arrays (ids id_base + i continue across it); a launch that also
    # writes the raw [5][n] state runs as one launch.  Both must give the same exits bit for
    # bit.
    binding = require_gpu()
    small = _small_limit()
    rnd = 4 * small
    m = binding.Model(inputs.pack_blob(inputs.random_weights(H, 25)), prec)
    for n in (rnd + 1, rnd + 777, 2 * rnd + small, 2 * rnd + small + 1, 2 * rnd + 2 * small,
              2 * rnd + 2 * small + 1):
        cond = inputs.transmission_conditions(n, 26)
        two = _exits(binding, m, cond, integ, K, raw=False)
        one = _exits(binding, m, cond, integ, K, raw=True)
        for k in one:
            np.testing.assert_array_equal(two[k], one[k], err_msg=f"n = {n}, {k}")
    m.close()


@pytest.mark.parametrize("prec,H", [("bf16", 512), ("fp8", 512), ("bf16", 256)])
def test_small_launch_matches_the_emulating_oracle(orc, prec, H):
    binding = require_gpu()
    n = 77
    cond = inputs.transmission_conditions(n, 23)
    w = inputs.random_weights(H, 24)
    m = binding.Model(inputs.pack_blob(w), prec)
    raw = _raw(binding, m, cond, "euler", 8).astype(np.float64)
    m.close()
    oprec = orc.PREC_BF16_EXP2 if prec == "bf16" else orc.PREC_FP8_EXP2
    ref = _oracle_raw(orc, w, cond, np.arange(n), 8, oprec, seed=7)
    err = np.abs(raw.T - ref).max(axis=1)
    print(f"{prec} H={H} small launch: p99 {np.quantile(err, 0.99):.2e} max {err.max():.2e}")
    if prec == "bf16":
        assert np.quantile(err, 0.99) < 1e-5 and err.max() < 5e-5
    else:
        assert np.quantile(err, 0.99) < 1e-4 and err.max() < 3e-4


@pytest.mark.parametrize("split,graphs,births", [(True, False, False), (False, True, False), (True, True, False),
                                                (False, False, True)])
def test_transport_does_not_depend_on_the_tile_choice(split, graphs, births):
    # Steps whose sample count only the device knows (the collided crossings of a first-flight
    # split step; a captured step's count below its bucket) choose the tile size on the device
    # when the host's bound exceeds 32 samples per compute unit; direct steps and births with
    # a count known on the host run a short last round on 32-sample tiles.  A bank that holds
    # every history at once takes every choice as the count falls; a bank of at most 32 x cu
    # slots only ever runs 32-sample tiles.  Histories draw their own random streams, so the
    # tallies agree up to the order of the FP64 tally additions.
    from paper_2512_13965_amd import transport
    binding = require_gpu()
    small = _small_limit()
    prob = inputs.checkerboard_problem(16, src=2)
    n = 5 * small                     # 4 x cu rounds of 128-sample tiles plus one of 32 samples per cu
    m = binding.Model(inputs.pack_blob(inputs.random_weights(256, 31, flags=2 if split else 0)), "bf16")
    src = binding.Model(inputs.pack_blob(inputs.random_weights(256, 32, n_in=12)), "bf16") if births else None
    out = {}
    for name, cap in (("large_bank", 8 * small), ("small_bank", small)):
        w = binding.World(cap, 1, 1 << 12)
        w.set_graphs(graphs)
        out[name] = transport.run_problem(w, prob, n, 5, binding.SAMPLER_GMC, m, 4, chunk=cap,
                                          source_model=src, source_K=3)
        w.close()
    m.close()
    if src is not None:
        src.close()
    a, b = out["large_bank"], out["small_bank"]
    print(f"split={split} graphs={graphs} births={births}: steps {a['steps']} / {b['steps']}, transmissions {a['transmissions']}")
    assert a["transmissions"] == b["transmissions"]
    for k in ("flux", "absorbed", "leak", "cutoff", "wpath", "path", "visits"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-12 * n, err_msg=k)
