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


# PREC_FP8_EXP2 (the FP8 sampler's order): fold_exp2's network with PREC_FP8's roundings, the
# activations entering an e4m3 layer halved before their rounding and that layer's sum doubled.

@pytest.mark.parametrize("H,K", [(128, 1), (256, 3)])
def test_fp8_exp2_without_its_roundings_is_the_plain_network(orc, monkeypatch, H, K):
    # with both rounding functions replaced by the identity only the float32 rounding of the
    # folded parameters remains: every factor (the fold's -log2(e) and -ln 2, the halving, the
    # doubling, the layer scales) has to cancel exactly for this to hold
    w = inputs.random_weights(H, 17)
    cond = inputs.transmission_conditions(48, 18)
    z = inputs.noise(48, 19).astype(np.float64)
    plain = orc.sample_raw(w, cond, K, z, orc.PREC_FP64)
    ident = lambda a: np.asarray(a, np.float64)
    monkeypatch.setattr(orc, "round_e4m3", ident)
    monkeypatch.setattr(orc, "round_bf16", ident)
    got = orc.sample_raw(w, cond, K, z, orc.PREC_FP8_EXP2)
    assert np.abs(got - plain).max() < 1e-7 * max(1.0, np.abs(plain).max())


def _saturation_case(orc):
    """10 -> 4 -> 4 -> 5: layer 1 (BF16) has no weights and bias 60 on row 0, so its folded
    pre-activation is a' = float32(60 * -log2(e)) = -86.5617... and its scaled activation
    a' / (1 + 2^a') is a' itself in FP64; layer 2 (e4m3, activation scale 2^-3, weight scale
    2^-4: W / sw = 16 on the diagonal) copies row 0; the output layer (BF16) copies row 0 into
    v0."""
    W = [np.zeros((4, 10), np.float32), np.eye(4, dtype=np.float32), np.zeros((5, 4), np.float32)]
    b = [np.array([60.0, 0, 0, 0], np.float32), np.zeros(4, np.float32), np.zeros(5, np.float32)]
    W[2][0, 0] = 1.0
    return inputs.Weights(4, W, b, np.array([1.0, 2.0 ** -3, 1.0], np.float32),
                          np.array([1.0, 2.0 ** -4, 1.0], np.float32))


def test_fp8_exp2_halves_before_rounding(orc):
    # worked by hand: a' = -86.5617 enters the e4m3 layer halved: -43.2809 / 2^-3 = -346.25,
    # which e4m3 (steps of 32 in [256, 448]) rounds to -352 (not saturated); the doubled sum is
    # -352 * 16 * 2 * 2^-3 * 2^-4 = -88, whose scaled activation is -88 again; the output
    # layer's weight is -ln 2 rounded to BF16, -0.69140625, so v0 = 88 * 0.69140625 = 60.84375.
    # Rounding the unhalved -692.49 would have saturated at -448 (v0 = 38.72 without the
    # doubling), and so would -43.28 divided by the weight scale instead (swapped scales).
    w = _saturation_case(orc)
    assert float(np.float32(60.0) * orc.NEG_LOG2E_F32) * 4 == pytest.approx(-346.247, abs=1e-3)
    v = orc.velocity(w, np.zeros((1, 5)), 0.0, np.zeros((1, 4)), orc.PREC_FP8_EXP2)
    assert v[0, 0] == 88 * 0.69140625
    np.testing.assert_array_equal(v[0, 1:], 0.0)


def test_fp8_exp2_rounds_other_values_than_fp8(orc):
    # the two FP8 evaluation orders round different values, and both stay within FP8's error
    # of the exact network
    w = inputs.random_weights(256, 21)
    cond = inputs.transmission_conditions(64, 22)
    z = inputs.noise(64, 23).astype(np.float64)
    exact = orc.sample_raw(w, cond, 4, z, orc.PREC_FP64)
    a = orc.sample_raw(w, cond, 4, z, orc.PREC_FP8)
    b = orc.sample_raw(w, cond, 4, z, orc.PREC_FP8_EXP2)
    assert np.abs(a - b).max() > 1e-4
    ea, eb = np.abs(a - exact).max(), np.abs(b - exact).max()
    assert eb < 3 * ea and ea < 3 * eb
