"""Statistical acceptance of the fitted residual network with adaptive modulation
(`weights/gmc_film_h512.bin`; paper "Network Architecture and Inputs"), BF16 on the GPU.

Parity unpinned (a learned law): the exit law against the FP64 oracle's analog walk (mode C)
at the same entry condition, and the mean-chord invariance E[l] = pi/4 (P3).  Measured with
RK4 x 12 at (tau, c) = (10, 1), (100, 1), (30, 0.95): face TV <= 0.0061, KS position <= 0.053,
exit cosine <= 0.0059, ln path <= 0.0114, E[l] within 2.5 % of pi/4 at tau = 1, 10, 100; with
Euler K = 16: face TV <= 0.0127, KS position <= 0.051, cosine <= 0.046, ln path <= 0.030 (the
plain MLP fitted on the same data: RK4 0.0070 / 0.073 / 0.0052 / 0.0128).  Budgets: these plus
the two-sample KS noise (0.0075 at 10^5 against 5 10^4 samples) and some room.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2512_13965_amd", "weights", "gmc_film_h512.bin")
BUDGET = {"rk4": (0.012, 0.07, 0.015, 0.02), "euler": (0.02, 0.065, 0.06, 0.04)}


def _fixed(n, tau, c, y, s):
    f = lambda v: np.full(n, np.float32(v))
    return inputs.Conditions(f(math.log(tau)), f(c), f(y), f(s))


@pytest.fixture(scope="module")
def trained():
    binding = require_gpu()
    if not os.path.exists(WEIGHTS):
        pytest.skip("no fitted residual network")
    m = binding.Model(open(WEIGHTS, "rb").read(), "bf16")
    yield binding, m
    m.close()


@pytest.mark.parametrize("integ,K", [("rk4", 12), ("euler", 16)])
@pytest.mark.parametrize("tau,c,y,s", [(10.0, 1.0, 0.3, 0.5), (100.0, 1.0, 0.5, -0.3), (30.0, 0.95, 0.9, -0.8)])
def test_exit_law_matches_the_walk(orc, trained, integ, K, tau, c, y, s):
    binding, m = trained
    n_g, n_o = 100_000, 50_000
    g = binding.gmc_sample(m, binding.DeviceCond.from_host(_fixed(n_g, tau, c, y, s)), integ, K, 5).to_host()
    o = orc.mc_transmit(_fixed(n_o, tau, c, y, s), 0, seed=17, nthreads=8)
    ok = g["face"] >= 0
    fg = np.bincount(g["face"][ok], minlength=4) / n_g
    fo = np.bincount(o["face"], minlength=4) / n_o
    tv = 0.5 * np.abs(fg - fo).sum()
    ks_pos = stats.ks_2samp(g["pos"][ok] + g["face"][ok], o["pos"] + o["face"]).statistic
    ks_cos = stats.ks_2samp(g["dir_cos"][ok], o["u"]).statistic
    ks_len = stats.ks_2samp(np.log(g["path"][ok]), np.log(o["len"])).statistic
    print(f"film {integ}x{K} tau={tau} c={c}: face TV {tv:.4f}, KS pos {ks_pos:.4f} cos {ks_cos:.4f} "
          f"ln l {ks_len:.4f}, rejected {1 - ok.mean():.2e}")
    b = BUDGET[integ]
    assert tv < b[0] and ks_pos < b[1] and ks_cos < b[2] and ks_len < b[3]
    assert ok.mean() > 1 - 1e-5


def test_rk4_mean_path_length_invariance(trained):
    binding, m = trained
    for tau in (1.0, 10.0, 100.0):
        cond = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(200_000, tau, 1.0, seed=3))
        g = binding.gmc_sample(m, cond, "rk4", 12, 9).to_host()
        rel = abs(g["path"].mean() - math.pi / 4) / (math.pi / 4)
        print(f"film rk4x12 tau={tau}: E[path] = {g['path'].mean():.4f}")
        assert rel < 0.04
