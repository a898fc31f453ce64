"""CPU checks of the training tool: the torch network it fits is the network the sampler and
the oracle evaluate (same layer order, input order and weight layout in the blob)."""
import numpy as np
import torch

from paper_2512_13965_amd import inputs
from paper_2512_13965_amd.train import VelocityMLP


def test_exported_weights_reproduce_the_torch_network(orc):
    torch.manual_seed(0)
    m = VelocityMLP(64).double()
    w = m.to_weights(seed=1, act_scale=[1.0] * 5)
    blob = inputs.unpack_blob(inputs.pack_blob(w))
    cond = inputs.transmission_conditions(32, seed=4)
    x = np.random.default_rng(1).standard_normal((32, 5))
    f = orc.condition_features(cond)
    ref = orc.velocity(blob, x, 0.3, f)
    with torch.no_grad():
        got = m(torch.from_numpy(x), torch.full((32,), 0.3, dtype=torch.float64),
                torch.from_numpy(f)).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6)   # blob stores float32 weights


def test_internal_model_export_reproduces_the_torch_network(orc):
    # the internal model's first layer reads [x (5), t, ln tau, c, 2x - 1, 2y - 1, cos, sin]
    torch.manual_seed(1)
    m = VelocityMLP(64, inputs.N_IN_INTERNAL).double()
    w = m.to_weights(seed=2, act_scale=[1.0] * 5)
    assert w.n_in == inputs.N_IN_INTERNAL
    blob = inputs.unpack_blob(inputs.pack_blob(w))
    assert blob.n_in == inputs.N_IN_INTERNAL
    cond = inputs.internal_conditions(32, seed=5)
    x = np.random.default_rng(2).standard_normal((32, 5))
    f = orc.condition_features(cond)
    ref = orc.velocity(blob, x, 0.7, f)
    with torch.no_grad():
        got = m(torch.from_numpy(x), torch.full((32,), 0.7, dtype=torch.float64),
                torch.from_numpy(f)).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6)
