"""Statistical acceptance of the fitted XY-geometry boundary model (entry and exit directions
are projections of directions on the sphere; paper eq. 1 and the condition's direction in the
unit disk of direction cosines).

Parity unpinned (a learned law): the exit law against the FP64 oracle's XY walk from the same
entry state, budgets = measured distances (BF16; Euler K = 32 and RK4 x 12) plus noise; and the
three-dimensional mean-chord invariance E[l] = 4 Area / Perimeter = 1 for isotropic incident
flux on a side of the unit square (pinned on the oracle in test_oracle_xy.py) on the model.
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
                       "paper_2512_13965_amd", "weights", "gmc_h512_xy.bin")
CASES = [(10.0, 1.0, 0.3, 0.8, 0.4), (100.0, 1.0, 0.5, 0.5, -0.6), (30.0, 0.95, 0.9, 0.3, -0.2),
         (10.0, 1.0, 0.5, 0.95, 0.0)]
# measured: Euler face TV <= 0.0097, KS pos <= 0.037, omega_x <= 0.024, omega_y <= 0.016, ln l <= 0.017;
#           RK4 x 12 face TV <= 0.0083, KS pos <= 0.099, omega_x <= 0.012, omega_y <= 0.009, ln l <= 0.010
# Euler KS pos at tau = 100: this model's position law there moves with the BF16 rounding of its
# first-layer weights (per-sample distance to the FP64 network 0.012-0.016): on 12,000 samples
# the FP64 network scores 0.046, BF16 with plain activations 0.042 and the sampler's order (hidden
# activations scaled by -log2(e), first-layer weights rounded after scaling) 0.060; measured on
# the GPU 0.056.  Budget: the FP64 network's 0.046 plus the spread of the rounding orders (0.015)
# plus the KS noise at these sample sizes (0.0075).
BUDGET = {"euler": (0.015, 0.07, 0.035, 0.025, 0.025), "rk4": (0.013, 0.13, 0.02, 0.015, 0.016)}


def _fixed(n, tau, c, y, ox, oy):
    f = lambda v: np.full(n, np.float32(v))
    return inputs.Conditions(f(math.log(tau)), f(c), f(y), f(oy), None, f(ox))


@pytest.fixture(scope="module")
def trained():
    binding = require_gpu()
    if not os.path.exists(WEIGHTS):
        pytest.skip("no fitted XY weights")
    m = binding.Model(open(WEIGHTS, "rb").read(), "bf16")
    yield binding, m
    m.close()


@pytest.mark.parametrize("integ,K", [("euler", 32), ("rk4", 12)])
@pytest.mark.parametrize("case", CASES)
def test_xy_exit_law_matches_the_walk(orc, trained, integ, K, case):
    binding, m = trained
    g = binding.gmc_sample(m, binding.DeviceCond.from_host(_fixed(100_000, *case)), integ, K, 5).to_host()
    o = orc.mc_transmit(_fixed(50_000, *case), 0, seed=17, nthreads=8)
    fg = np.bincount(g["face"], minlength=4) / 100_000
    fo = np.bincount(o["face"], minlength=4) / 50_000
    tv = 0.5 * np.abs(fg - fo).sum()
    ks = [stats.ks_2samp(g["pos"] + g["face"], o["pos"] + o["face"]).statistic,
          stats.ks_2samp(g["dir_cos"], o["u"]).statistic, stats.ks_2samp(g["dir_sin"], o["v"]).statistic,
          stats.ks_2samp(np.log(g["path"]), np.log(o["len"])).statistic]
    print(f"{integ}x{K} {case}: face TV {tv:.4f} KS pos/ox/oy/lnl {[round(k, 4) for k in ks]}")
    b = BUDGET[integ]
    assert tv < b[0] and ks[0] < b[1] and ks[1] < b[2] and ks[2] < b[3] and ks[3] < b[4]
    assert np.all(g["dir_cos"] ** 2 + g["dir_sin"] ** 2 <= 1.0 + 1e-5)


def test_xy_mean_chord_invariance_on_the_fitted_model(trained):
    # RK4 x 12 measured 1.0003 / 0.9958 / 1.0107 at tau = 1 / 10 / 100
    binding, m = trained
    for tau in (1.0, 10.0, 100.0):
        g = binding.gmc_sample(m, binding.DeviceCond.from_host(inputs.fixed_xy_conditions(200_000, tau, 1.0, 3)),
                               "rk4", 12, 9).to_host()
        print(f"tau {tau}: E[l] = {g['path'].mean():.4f}")
        assert abs(g["path"].mean() - 1.0) < 0.02
