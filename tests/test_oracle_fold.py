"""Pins of the oracle's exp2-folded evaluation order (PREC_BF16_EXP2: BF16 operands, hidden
activations carried scaled by -log2(e), the order of the library's BF16 sampler).  It is
PREC_BF16's operand rounding (pinned in test_oracle_quant.py) applied to the network of
fold_exp2, so what is pinned here is that fold_exp2 with its activation is the same network:
closed forms of the scaled activation, agreement with the plain network in FP64 to the float32
rounding of the folded parameters, the hand-worked value of the hand-built network, and which
values the folded order rounds."""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs
from tests import quant_case


def test_scaled_activation_closed_form(orc):
    for x in (-30.0, -2.5, -0.3, 0.0, 0.7, 4.0, 40.0):
        silu = x / (1.0 + math.exp(-x))
        a = -x / math.log(2.0)
        assert orc.silu_exp2(np.array([a]))[0] == pytest.approx(-silu / math.log(2.0), rel=1e-14, abs=1e-300)


def test_constants_are_the_float32_values_of_minus_log2e_and_minus_ln2(orc):
    assert orc.NEG_LOG2E_F32.dtype == np.float32 and orc.NEG_LN2_F32.dtype == np.float32
    assert abs(float(orc.NEG_LOG2E_F32) + 1.4426950408889634) < 2 ** -23
    assert abs(float(orc.NEG_LN2_F32) + 0.6931471805599453) < 2 ** -24
    # their product is 1 to float32 accuracy: the output layer undoes the first layer's factor
    assert abs(float(orc.NEG_LOG2E_F32) * float(orc.NEG_LN2_F32) - 1.0) < 2 ** -22


@pytest.mark.parametrize("H,K", [(128, 1), (256, 4)])
def test_folded_network_is_the_plain_network(orc, H, K):
    w = inputs.random_weights(H, 7)
    cond = inputs.transmission_conditions(64, 8)
    z = inputs.noise(64, 9).astype(np.float64)
    plain = orc.sample_raw(w, cond, K, z, orc.PREC_FP64)
    folded = orc.sample_raw(orc.fold_exp2(w), cond, K, z, orc.PREC_FP64)
    # only the float32 rounding of the folded parameters (2^-24 relative) separates the two
    assert np.abs(folded - plain).max() < 1e-7 * max(1.0, np.abs(plain).max())
    # a fold with the two factors swapped is a different network
    bad = orc.fold_exp2(w)
    bad.W[0] = np.asarray(w.W[0], np.float32) * orc.NEG_LN2_F32
    assert np.abs(orc.sample_raw(bad, cond, K, z, orc.PREC_FP64) - plain).max() > 1e-3


def test_folded_hand_network_gives_the_hand_worked_value(orc):
    # the hand-built network of tests/quant_case.py in FP64: x_1 is the literal worked out by
    # hand, to the float32 rounding of the folded parameters
    w = quant_case.network(16)
    x1 = orc.sample_raw(orc.fold_exp2(w), quant_case.conditions(2), 1, quant_case.noise(2), orc.PREC_FP64)
    np.testing.assert_allclose(x1, np.repeat(quant_case.EXPECTED["fp32"][None, :], 2, axis=0), rtol=1e-6)


def test_bf16_exp2_rounds_the_scaled_values(orc):
    # the folded first-layer weight 1024 is -1024 log2(e) rounded to BF16 (-1024 (1 + 57/128)),
    # not -log2(e) times the rounded weight
    w = quant_case.network(16)
    f = orc.fold_exp2(w)
    rd = lambda v: float(orc.round_bf16(np.array([v]))[0])
    assert rd(f.W[0][0, 0]) == rd(np.float32(1024.0) * orc.NEG_LOG2E_F32) == -1024 * 1.4453125
    assert rd(orc.NEG_LOG2E_F32) == -1.4453125
    # the two BF16 evaluation orders differ; the exact network is the same
    cond, z = quant_case.conditions(1), quant_case.noise(1)
    a = orc.sample_raw(w, cond, 1, z, orc.PREC_BF16)
    b = orc.sample_raw(w, cond, 1, z, orc.PREC_BF16_EXP2)
    assert np.abs(a - b).max() > 1e-4
