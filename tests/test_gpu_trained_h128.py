"""Statistical acceptance of the fitted boundary model of width H = 128 (the network the
sampler runs fastest, used to place GMC against the analog walk in optically thick cells; fitted
on cells up to tau = 1000).

Parity unpinned (a learned model): the reference is the FP64 oracle's analog walk (mode C) at
the same entry condition, with the paper's integrator (classic RK4, 12 steps).  Budgets are the
measured distances plus sampling noise; measured: face TV <= 0.012, KS cos <= 0.011, KS ln l
<= 0.014; KS position <= 0.06 up to tau = 100, <= 0.15 at tau = 300 and <= 0.36 at tau = 1000
(the exit position of a reflection from a very thick cell is sharply peaked at the entry point,
which the flow smears: the loosest fit, also for the H = 512 model, 0.15 at tau = 300); E[l]
within 5 % of pi / 4 at tau = 10, 100, 300, 1000.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_2512_13965_amd import inputs
from tests.gpu_util import drop_rejected, require_gpu

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2512_13965_amd", "weights", "gmc_h128.bin")


def _fixed(n, tau, c, y, s):
    f = lambda v: np.full(n, np.float32(v))
    return inputs.Conditions(f(math.log(tau)), f(c), f(y), f(s))


@pytest.fixture(scope="module")
def trained():
    binding = require_gpu()
    if not os.path.exists(WEIGHTS):
        pytest.skip("no fitted weights")
    m = binding.Model(open(WEIGHTS, "rb").read(), "bf16")
    assert m.hidden == 128
    yield binding, m
    m.close()


@pytest.mark.parametrize("tau,c,y,s,pos_budget", [(10.0, 1.0, 0.3, 0.5, 0.1), (100.0, 1.0, 0.5, -0.3, 0.1),
                                                  (30.0, 0.95, 0.9, -0.8, 0.1), (300.0, 1.0, 0.5, 0.2, 0.2),
                                                  (300.0, 0.99, 0.2, -0.6, 0.2), (1000.0, 1.0, 0.5, 0.0, 0.32),
                                                  (1000.0, 0.999, 0.8, 0.5, 0.42)])
def test_h128_exit_law_matches_the_walk(orc, trained, tau, c, y, s, pos_budget):
    binding, m = trained
    n_g, n_o = 100_000, (20_000 if tau > 500 else 50_000)
    g = drop_rejected(binding.gmc_sample(m, binding.DeviceCond.from_host(_fixed(n_g, tau, c, y, s)), "rk4",
                                         12, 5).to_host())
    o = orc.mc_transmit(_fixed(n_o, tau, c, y, s), 0, seed=17, nthreads=8)
    fg = np.bincount(g["face"], minlength=4) / len(g["face"])
    fo = np.bincount(o["face"], minlength=4) / n_o
    tv_face = 0.5 * np.abs(fg - fo).sum()
    ks_cos = stats.ks_2samp(g["dir_cos"], o["u"]).statistic
    ks_len = stats.ks_2samp(np.log(g["path"]), np.log(o["len"])).statistic
    ks_pos = stats.ks_2samp(g["pos"] + g["face"], o["pos"] + o["face"]).statistic
    print(f"H=128 rk4x12 tau={tau} c={c}: face TV {tv_face:.4f}, KS pos {ks_pos:.4f} cos {ks_cos:.4f} "
          f"ln l {ks_len:.4f}")
    assert tv_face < 0.025
    assert ks_cos < 0.02 and ks_len < 0.02 and ks_pos < pos_budget


def test_h128_mean_chord_invariance(trained):
    # P3: E[path] = pi / 4 at c = 1 for every tau
    binding, m = trained
    for tau in (10.0, 100.0, 300.0, 1000.0):
        cond = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(200_000, tau, 1.0, seed=3))
        g = drop_rejected(binding.gmc_sample(m, cond, "rk4", 12, 9).to_host())
        rel = abs(g["path"].mean() - math.pi / 4) / (math.pi / 4)
        print(f"H=128 rk4x12 tau={tau}: E[path] = {g['path'].mean():.4f}")
        assert rel < 0.065
