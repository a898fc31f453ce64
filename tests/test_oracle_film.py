"""Pins of the oracle's residual network with adaptive modulation (paper "Network Architecture
and Inputs": learned embeddings of t and c, residual blocks modulated by the physical context;
the layer details are the library's reading of a section whose specification is missing).

Each pin checks the oracle against something other than its own formula: values worked out by
hand (time features, a modulated block, a rounding tie of the bfloat16 residual stream),
closed forms of the sampler ODE (constant and time-only fields), the reduction of identity
blocks to one affine map, and a separate torch evaluation of the unmodulated residual MLP."""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs
from tests import film_case


def _cond(n, seed=3, n_in=10):
    if n_in == 12:
        return inputs.internal_conditions(n, seed)
    return inputs.transmission_conditions(n, seed)


def test_time_features_hand_values(orc):
    r = math.sqrt(0.5)
    np.testing.assert_allclose(orc.time_features(0.0), [0, 1, 0, 1, 0, 1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(orc.time_features(0.5), [1, 0, 0, -1, 0, 1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(orc.time_features(0.25), [r, r, 1, 0, 0, -1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(orc.time_features(1.0), [0, -1, 0, 1, 0, 1, 0, 1], atol=1e-15)


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
@pytest.mark.parametrize("integ,K", [("euler", 1), ("euler", 3), ("rk4", 2)])
def test_constant_field_moves_z_by_the_bias(orc, prec, integ, K):
    b = np.array([0.5, -1.25, 2.0, 0.75, -0.5])
    w = film_case.constant(b)
    z = inputs.noise(6, 4)
    f = orc.sample_raw_rk4 if integ == "rk4" else orc.sample_raw
    got = f(w, _cond(6), K, z, prec)
    np.testing.assert_allclose(got, z.T.astype(np.float64) + b, rtol=0, atol=1e-14)


def test_time_probe_integrates_the_time_features(orc):
    # v = (sin pi t, cos pi t, cos 8 pi t): Euler sums f(k/K)/K, RK4 takes Simpson's rule
    # per step (a field of t only)
    w = film_case.time_probe()
    z = np.zeros((5, 2))
    f = [lambda t: math.sin(math.pi * t), lambda t: math.cos(math.pi * t), lambda t: math.cos(8 * math.pi * t)]
    K = 5
    eul = orc.sample_raw(w, _cond(2), K, z)
    rk = orc.sample_raw_rk4(w, _cond(2), K, z)
    h = 1.0 / K
    for d in range(3):
        e = sum(f[d](k * h) for k in range(K)) * h
        s = sum(h / 6 * (f[d](k * h) + 4 * f[d](k * h + h / 2) + f[d](k * h + h)) for k in range(K))
        np.testing.assert_allclose(eul[:, d], e, rtol=0, atol=1e-14)
        np.testing.assert_allclose(rk[:, d], s, rtol=0, atol=1e-14)
    # with many RK4 steps the integrals of sin(pi t), cos(pi t), cos(8 pi t) over [0, 1]
    rk = orc.sample_raw_rk4(w, _cond(1), 64, np.zeros((5, 1)))
    np.testing.assert_allclose(rk[0, :3], [2 / math.pi, 0.0, 0.0], atol=1e-8)


def test_modulated_block_by_hand(orc):
    # H = 4, E = 2, one block.  h0 = x[:4]; e = SiLU(b_e) = (SiLU(0), SiLU(64)) = (0, 64);
    # main map 2 I + (0, 1, 0, -1); scale 1 + G e = (1, 2, 0, 1.5); shift S e = (0, .5, 2, -1)
    x = np.array([[1.0, -2.0, 0.5, 3.0, 0.7]])
    dims = inputs.film_layer_dims(4, 2, 10, 1)
    W = [np.zeros(d, np.float32) for d in dims]
    b = [np.zeros(d[0], np.float32) for d in dims]
    W[0][:4, :4] = np.eye(4)
    b[1][:] = [0.0, 64.0]
    W[2][:] = 2 * np.eye(4)
    b[2][:] = [0.0, 1.0, 0.0, -1.0]
    W[3][:, 1] = [0.0, 1 / 64, -1 / 64, 1 / 128]
    W[4][:, 1] = [0.0, 1 / 128, 1 / 32, -1 / 64]
    W[5][:4, :4] = np.eye(4)
    w = inputs.FilmWeights(4, 2, W, b)
    v = orc.velocity(w, x, 0.0, np.zeros((1, 4)))
    silu = lambda a: a / (1 + math.exp(-a))
    # pre-activations (2*1 + 0) * 1 + 0, (2*-2 + 1) * 2 + .5, (2*.5) * 0 + 2, (2*3 - 1) * 1.5 - 1
    want = [1 + silu(2.0), -2 + silu(-5.5), 0.5 + silu(2.0), 3 + silu(6.5), 0.0]
    np.testing.assert_allclose(v[0], want, rtol=1e-15, atol=1e-15)


def test_identity_blocks_reduce_to_one_affine_map(orc):
    # zero main maps and shifts: every branch is SiLU(scale * 0 + 0) = 0 whatever the (random)
    # modulation, so v = W_o (W_in u + b_in) + b_o = (W_o W_in) u + (W_o b_in + b_o)
    w = inputs.random_film_weights(64, 11, emb=32, blocks=3)
    for j in range(3):
        w.W[2 + 3 * j][:] = 0
        w.b[2 + 3 * j][:] = 0
        w.W[4 + 3 * j][:] = 0
        w.b[4 + 3 * j][:] = 0
    g = inputs.rng(2)
    x = g.normal(size=(7, 5))
    condf = g.normal(size=(7, 4))
    t = 0.3
    v = orc.velocity(w, x, t, condf)
    u = np.concatenate([x, np.tile(orc.time_features(t), (7, 1)), condf], axis=1)
    Wi, Wo = w.W[0].astype(np.float64), w.W[-1].astype(np.float64)
    M = Wo @ Wi
    c0 = Wo @ w.b[0].astype(np.float64) + w.b[-1]
    np.testing.assert_allclose(v, u @ M.T + c0, rtol=1e-12, atol=1e-13)


def test_unmodulated_network_is_the_plain_residual_mlp(orc):
    # zero scale and shift maps (weights and biases): each block is h + SiLU(A h + a), here
    # evaluated separately with torch in float64
    torch = pytest.importorskip("torch")
    F = torch.nn.functional
    w = inputs.random_film_weights(64, 12, emb=32, blocks=3, n_in=12)
    for j in range(3):
        for l in (3 + 3 * j, 4 + 3 * j):
            w.W[l][:] = 0
            w.b[l][:] = 0
    g = inputs.rng(3)
    x = g.normal(size=(9, 5))
    condf = g.normal(size=(9, 6))
    t = 0.625
    v = orc.velocity(w, x, t, condf)
    T = lambda a: torch.tensor(np.asarray(a, np.float64))
    ang = [math.pi * 2 ** j * t for j in range(4)]
    phi = T([[f(a) for a in ang for f in (math.sin, math.cos)]]).repeat(9, 1)
    h = F.linear(torch.cat([T(x), phi, T(condf)], 1), T(w.W[0]), T(w.b[0]))
    for j in range(3):
        h = h + F.silu(F.linear(h, T(w.W[2 + 3 * j]), T(w.b[2 + 3 * j])))
    ref = F.linear(h, T(w.W[-1]), T(w.b[-1])).numpy()
    np.testing.assert_allclose(v, ref, rtol=1e-12, atol=1e-13)


def test_condition_reaches_the_output_only_through_its_paths(orc):
    # with the input layer's condition columns zeroed, the condition acts only through the
    # embedding; zeroing the scale and shift maps as well makes v independent of it
    w = inputs.random_film_weights(64, 13)
    w.W[0][:, 13:] = 0
    g = inputs.rng(4)
    x = g.normal(size=(5, 5))
    c1, c2 = g.normal(size=(5, 4)), g.normal(size=(5, 4))
    assert np.abs(orc.velocity(w, x, 0.4, c1) - orc.velocity(w, x, 0.4, c2)).max() > 1e-3
    for j in range(3):
        for l in (3 + 3 * j, 4 + 3 * j):
            w.W[l][:] = 0
    np.testing.assert_array_equal(orc.velocity(w, x, 0.4, c1), orc.velocity(w, x, 0.4, c2))


@pytest.mark.parametrize("prec,key", [("fp64", "fp32"), ("bf16", "bf16")])
def test_bf16_residual_stream_rounds_to_even(orc, prec, key):
    w = film_case.residual_tie()
    z = np.zeros((5, 3))
    z[0] = film_case.RESIDUAL_TIE_Z0
    z[1:] = [[0.5], [-0.25], [2.0], [-1.0]]
    got = orc.sample_raw(w, _cond(3), 1, z, prec)
    np.testing.assert_array_equal(got[:, 0], film_case.RESIDUAL_TIE_X1[key])
    np.testing.assert_array_equal(got[:, 1:], z[1:].T)


def test_fp8_is_not_a_precision_of_the_residual_network(orc):
    w = film_case.constant(np.zeros(5))
    with pytest.raises(ValueError):
        orc.velocity(w, np.zeros((1, 5)), 0.0, np.zeros((1, 4)), orc.PREC_FP8)


def test_blob_round_trip():
    w = inputs.random_film_weights(128, 5, n_in=11, flags=1)
    w2 = inputs.unpack_blob(inputs.pack_blob(w))
    assert isinstance(w2, inputs.FilmWeights)
    assert (w2.hidden, w2.emb, w2.blocks, w2.n_in, w2.flags) == (128, 32, 3, 11, 5)
    for a, b in zip(w.W + w.b, w2.W + w2.b):
        np.testing.assert_array_equal(a, b)
