"""A hand-built velocity network whose outputs are worked out by hand, for pinning where the
BF16 and FP8 e4m3 operand roundings happen (the oracle's quantisation emulation and the
kernels alike).

Every weight is a power of two or a small dyadic number, every pre-activation after the first
layer is an integer in [37, 256] or exactly 0, so SiLU(a) = a / (1 + e^-a) is the identity
(e^-37 < 2^-53) or 0 in FP64 and in FP32, and every sum is exact.  Only the roundings of the
operands change the values, so the result of one Euler step (K = 1, t = 0) from a given z is a
literal.  The ties are placed as follows (BF16 keeps 8 significant bits, e4m3 4):

layer 1 (10 -> H, BF16 operands in every quantised precision)
  row 0: 1024 * x0 - 984,  x0 = 1 + 2^-8: BF16 tie, to even 1      -> 40 (unrounded 44)
  row 1: 1024 * ln tau - 984, ln tau = 1 + 3 * 2^-8: tie, to 1 + 2^-6 -> 56 (unrounded 52)
  row 2: 1028 * x1 - 984,  x1 = 1: the weight 1028 = 1024 (1 + 2^-8) ties to 1024 -> 40 (44)
  row 3: 128 * (2 y_in - 1) - 24, y_in = 3/4                       -> 40 (input order)
  row 5: 4 * c + 40, c = 1/2                                       -> 42
  row 6: 400 * c                                                    -> 200
  row 7: 1024 * t + 40                                              -> 40 at t = 0
layer 2 (H -> H; FP8: act_scale 2^-1, w_scale 2^-4)
  rows 0, 1, 2, 5, 6, 7 copy their input, row 3 = 1.0625 * h3, row 4 = 4 * h0.
  FP8: h / 2^-1 -> e4m3: 42 -> 84 ties to 80 (-> 40); 200 -> 400 ties to 384 (-> 192);
  1.0625 / 2^-4 = 17 ties to 16 (weight 1.0); BF16 keeps 42, 200 and 1.0625.
  With the two scales swapped, 40 / 2^-4 = 640 would saturate at 448 (row 0 -> 28).
layers 3, 4 (H -> H; FP8 scales 1): identity on rows 0..7.
layer 5 (H -> 5, BF16):
  v0 = h0 / 32, v1 = h1 / 32, v2 = h2 / 32 + h3 / 64, v3 = h4 / 128 + h5 / 64,
  v4 = h6 / 256 + h7 / 1024 + (1/8 + 2^-20)   (the bias is not rounded: BF16 or e4m3 would
  drop the 2^-20)
z = (1 + 2^-8, 1, 0, 0, 0); x_1 = z + v.
"""
from __future__ import annotations

import numpy as np

from paper_2512_13965_amd import inputs

Z = np.array([1.0 + 2.0 ** -8, 1.0, 0.0, 0.0, 0.0])
LOG_TAU = 1.0 + 3.0 * 2.0 ** -8
C = 0.5
Y_IN = 0.75
SIN_TH = 0.0
BIAS5 = 0.125 + 2.0 ** -20

# x_1 after one Euler step at t = 0, worked out by hand (see the module docstring)
EXPECTED = {
    # no rounding: rows 0, 1, 2 keep 44, 52, 44; row 3 = 42.5, row 5 = 42, row 6 = 200
    "fp32": np.array([1.00390625 + 44 / 32, 1.0 + 52 / 32, 44 / 32 + 42.5 / 64,
                      176 / 128 + 42 / 64, 200 / 256 + 40 / 1024 + BIAS5]),
    # BF16 operands: ties resolved to 40, 56, 40; 42, 200 and the weight 1.0625 exact
    "bf16": np.array([1.00390625 + 40 / 32, 1.0 + 56 / 32, 40 / 32 + 42.5 / 64,
                      160 / 128 + 42 / 64, 200 / 256 + 40 / 1024 + BIAS5]),
    # FP8 hidden layers: additionally 42 -> 40, 200 -> 192, weight 1.0625 -> 1
    "fp8": np.array([1.00390625 + 40 / 32, 1.0 + 56 / 32, 40 / 32 + 40 / 64,
                     160 / 128 + 40 / 64, 192 / 256 + 40 / 1024 + BIAS5]),
}


def network(H: int = 128) -> inputs.Weights:
    """The hand-built 10 -> H x4 -> 5 network (H >= 8); unused rows are zero with zero bias."""
    W = [np.zeros((H, 10), np.float32), np.zeros((H, H), np.float32), np.zeros((H, H), np.float32),
         np.zeros((H, H), np.float32), np.zeros((5, H), np.float32)]
    b = [np.zeros(H, np.float32), np.zeros(H, np.float32), np.zeros(H, np.float32),
         np.zeros(H, np.float32), np.zeros(5, np.float32)]
    # layer 1: input columns [x0..x4, t, ln tau, c, 2 y_in - 1, sin th]
    W[0][0, 0], b[0][0] = 1024.0, -984.0
    W[0][1, 6], b[0][1] = 1024.0, -984.0
    W[0][2, 1], b[0][2] = 1028.0, -984.0
    W[0][3, 8], b[0][3] = 128.0, -24.0
    W[0][5, 7], b[0][5] = 4.0, 40.0
    W[0][6, 7] = 400.0
    W[0][7, 5], b[0][7] = 1024.0, 40.0
    # layer 2
    for r in (0, 1, 2, 5, 6, 7):
        W[1][r, r] = 1.0
    W[1][3, 3] = 1.0625
    W[1][4, 0] = 4.0
    # layers 3 and 4: identity on rows 0..7
    for l in (2, 3):
        for r in range(8):
            W[l][r, r] = 1.0
    # layer 5
    W[4][0, 0] = 1 / 32
    W[4][1, 1] = 1 / 32
    W[4][2, 2], W[4][2, 3] = 1 / 32, 1 / 64
    W[4][3, 4], W[4][3, 5] = 1 / 128, 1 / 64
    W[4][4, 6], W[4][4, 7] = 1 / 256, 1 / 1024
    b[4][4] = BIAS5
    act = np.array([1.0, 0.5, 1.0, 1.0, 1.0], np.float32)
    wsc = np.array([1.0, 2.0 ** -4, 1.0, 1.0, 1.0], np.float32)
    return inputs.Weights(H, W, b, act, wsc, seed=0)


def conditions(n: int = 1) -> inputs.Conditions:
    f = lambda v: np.full(n, v, np.float32)
    return inputs.Conditions(f(LOG_TAU), f(C), f(Y_IN), f(SIN_TH))


def noise(n: int = 1) -> np.ndarray:
    """z of every sample, layout [5][n] (float32; every value exact)."""
    return np.repeat(Z[:, None], n, axis=1).astype(np.float32)
