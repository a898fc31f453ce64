"""Statistical acceptance of the fitted boundary model for rectangular cells (paper eq. 10: the
condition carries the optical width and height; here ln tau of the entry face and ln A,
A = width / entry-face length, fitted for A in [1/4, 4]).

Parity unpinned (a learned law): the exit law is compared with the FP64 oracle's analog walk
from the same entry state; budgets are the measured distances (BF16; Euler K = 32 and RK4 x 12)
plus sampling noise.  The mean-chord invariance split by entry side,
E(A; tau) + A^2 E(1/A; tau A) = pi A / 2 (pinned on the oracle in test_oracle_rect.py), is
checked on the fitted model, and a 112 x 56 lattice of 1/16 x 1/8 cm cells is transported at
the statistical floor of analog MC.
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
                       "paper_2512_13965_amd", "weights", "gmc_h512_rect.bin")
CASES = [(10.0, 1.0, 0.5, 0.3, 0.5), (10.0, 1.0, 2.0, 0.5, -0.3), (50.0, 0.95, 0.3, 0.8, -0.6),
         (30.0, 1.0, 3.5, 0.2, 0.1), (100.0, 1.0, 1.0, 0.5, 0.0)]
# measured: Euler face TV <= 0.0094, KS pos <= 0.031, cos <= 0.026, ln l <= 0.017;
#           RK4 x 12 face TV <= 0.0122, KS pos <= 0.053, cos <= 0.010, ln l <= 0.0082
BUDGET = {"euler": (0.015, 0.045, 0.04, 0.025), "rk4": (0.02, 0.08, 0.02, 0.015)}


def _fixed(n, tau, c, A, y, s):
    f = lambda v: np.full(n, np.float32(v))
    return inputs.Conditions(f(math.log(tau)), f(c), f(y), f(s), f(math.log(A)))


@pytest.fixture(scope="module")
def trained():
    binding = require_gpu()
    if not os.path.exists(WEIGHTS):
        pytest.skip("no fitted rectangular-cell weights")
    m = binding.Model(open(WEIGHTS, "rb").read(), "bf16")
    assert m.n_in == 11
    yield binding, m
    m.close()


@pytest.mark.parametrize("integ,K", [("euler", 32), ("rk4", 12)])
@pytest.mark.parametrize("case", CASES)
def test_rect_exit_law_matches_the_walk(orc, trained, integ, K, case):
    binding, m = trained
    g = binding.gmc_sample(m, binding.DeviceCond.from_host(_fixed(100_000, *case)), integ, K, 5).to_host()
    o = orc.mc_transmit(_fixed(50_000, *case), 0, seed=17, nthreads=8)
    fg = np.bincount(g["face"], minlength=4) / 100_000
    fo = np.bincount(o["face"], minlength=4) / 50_000
    tv = 0.5 * np.abs(fg - fo).sum()
    ks_pos = stats.ks_2samp(g["pos"] + g["face"], o["pos"] + o["face"]).statistic
    ks_cos = stats.ks_2samp(g["dir_cos"], o["u"]).statistic
    ks_len = stats.ks_2samp(np.log(g["path"]), np.log(o["len"])).statistic
    print(f"{integ}x{K} {case}: face TV {tv:.4f} KS pos {ks_pos:.4f} cos {ks_cos:.4f} ln l {ks_len:.4f}")
    b = BUDGET[integ]
    assert tv < b[0] and ks_pos < b[1] and ks_cos < b[2] and ks_len < b[3]


@pytest.mark.parametrize("tau,A", [(10.0, 2.0), (30.0, 0.5)])
def test_rect_mean_chord_invariance_on_the_fitted_model(trained, tau, A):
    # RK4 x 12 measured 3.1298 vs pi (A = 2) and 0.7838 vs pi / 4 (A = 1/2)
    binding, m = trained
    n = 200_000
    ca = inputs.fixed_cell_conditions(n, tau, 1.0, 3)
    cb = inputs.fixed_cell_conditions(n, tau * A, 1.0, 4)
    a = binding.gmc_sample(m, binding.DeviceCond.from_host(inputs.Conditions(
        ca.log_tau, ca.c, ca.y_in, ca.sin_th, np.full(n, np.float32(math.log(A))))), "rk4", 12, 9).to_host()
    b = binding.gmc_sample(m, binding.DeviceCond.from_host(inputs.Conditions(
        cb.log_tau, cb.c, cb.y_in, cb.sin_th, np.full(n, np.float32(-math.log(A))))), "rk4", 12, 10).to_host()
    lhs = a["path"].mean() + A * A * b["path"].mean()
    print(f"tau {tau} A {A}: {lhs:.4f} vs pi A / 2 = {math.pi * A / 2:.4f}")
    assert abs(lhs - math.pi * A / 2) < 0.015 * math.pi * A / 2


def test_rect_lattice_transport_at_the_statistical_floor(trained):
    # 112 x 56 cells of 1/16 x 1/8 cm (the lattice's cross sections): measured GMC RK4 x 12 vs
    # MC 0.0185, MC vs MC 0.0183 at 2e5 histories
    binding, m = trained
    from paper_2512_13965_amd import transport
    prob = inputs.lattice_problem(16, 8)
    n = 100_000
    w = binding.World(1 << 18, 1, 1 << 14)
    mc1 = transport.run_problem(w, prob, n, 1, binding.SAMPLER_MC)
    mc2 = transport.run_problem(w, prob, n, 2, binding.SAMPLER_MC)
    gm = transport.run_problem(w, prob, n, 3, binding.SAMPLER_GMC, m, 12, integrator="rk4")
    w.close()
    l1 = lambda a, b: np.abs(a["flux"] - b["flux"]).sum() / np.abs(b["flux"]).sum()
    floor, err = l1(mc2, mc1), l1(gm, mc1)
    print(f"rect lattice: GMC vs MC {err:.4f}, MC vs MC {floor:.4f}")
    assert err < 1.25 * floor
    assert abs(gm["absorbed"].sum() + gm["leak"].sum() + gm["cutoff"].sum() - n) < 1e-9 * n
