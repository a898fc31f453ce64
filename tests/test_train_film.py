"""The training module of the residual network (train.VelocityFiLM) computes the network the
sampler kernel and the oracle define, and exports weights whose blob round-trips (CPU)."""
import numpy as np
import pytest

from paper_2512_13965_amd import inputs

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n_in", [10, 11, 12])
def test_module_matches_the_oracle_on_its_exported_weights(orc, n_in):
    from paper_2512_13965_amd import train
    torch.manual_seed(n_in)
    m = train.VelocityFiLM(64, n_in).double()
    with torch.no_grad():
        for lin in m.layers:
            lin.weight.normal_(0.0, 0.3)
            lin.bias.normal_(0.0, 0.3)
    w = inputs.unpack_blob(inputs.pack_blob(m.to_weights(1)))
    assert isinstance(w, inputs.FilmWeights) and w.n_in == n_in and w.emb == inputs.FILM_EMB
    g = inputs.rng(n_in)
    x = g.normal(size=(7, 5))
    c = g.normal(size=(7, n_in - 6))
    t = 0.3
    ref = orc.velocity(w, x, t, c)
    # the module evaluated on the float32-rounded weights the blob holds
    with torch.no_grad():
        for lin, W, b in zip(m.layers, w.W, w.b):
            lin.weight.copy_(torch.from_numpy(W.astype(np.float64)))
            lin.bias.copy_(torch.from_numpy(b.astype(np.float64)))
    got = m(torch.from_numpy(x), torch.full((7,), t, dtype=torch.float64), torch.from_numpy(c)).detach().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_modulation_starts_at_zero():
    from paper_2512_13965_amd import train
    m = train.VelocityFiLM(64, 10)
    for j in range(m.blocks):
        for l in (3 + 3 * j, 4 + 3 * j):
            assert float(m.layers[l].weight.abs().max()) == 0.0 and float(m.layers[l].bias.abs().max()) == 0.0
