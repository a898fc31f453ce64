"""The kernels on the hand-built network of tests/quant_case.py: one Euler step from a given
z must reproduce, bit for bit, the values worked out by hand for FP32 operands.  The BF16 and
FP8 samplers evaluate the network with its hidden activations scaled by -log2(e) (the oracle's
PREC_BF16_EXP2 and PREC_FP8_EXP2), whose folded parameters are no longer dyadic: they are held
to that emulation of the same hand-built network (the exact sums there leave only the FP32
rounding of the bias additions, 1e-6 relative)."""
import numpy as np
import pytest
import torch

from paper_2512_13965_amd import inputs
from tests import quant_case
from tests.gpu_util import require_gpu

CASES = [("fp32", 128), ("fp32", 256), ("bf16", 128), ("bf16", 256), ("bf16", 512),
         ("fp8", 128), ("fp8", 256), ("fp8", 512)]


@pytest.mark.gpu
@pytest.mark.parametrize("prec,H", CASES)
def test_hand_network_exact_on_gpu(prec, H):
    binding = require_gpu()
    n = 300                                       # several tiles and a ragged tail
    m = binding.Model(inputs.pack_blob(quant_case.network(H)), prec)
    cond = binding.DeviceCond.from_host(quant_case.conditions(n))
    z = torch.from_numpy(quant_case.noise(n)).cuda().contiguous()
    raw = torch.empty(5 * n, dtype=torch.float32, device="cuda")
    binding.gmc_transmit(m, cond, 1, seed=1, id_base=0, noise=z, raw=raw)
    torch.cuda.synchronize()
    got = raw.view(5, n).cpu().numpy().T
    if prec in ("bf16", "fp8"):
        import oracle
        oprec = oracle.PREC_BF16_EXP2 if prec == "bf16" else oracle.PREC_FP8_EXP2
        ref = oracle.sample_raw(quant_case.network(H), quant_case.conditions(1), 1,
                                quant_case.noise(1).astype(np.float64), oprec)[0]
        np.testing.assert_allclose(got, np.repeat(ref[None, :], n, axis=0), rtol=1e-6, atol=1e-6)
        m.close()
        return
    want = quant_case.EXPECTED[prec].astype(np.float32)
    assert np.array_equal(want.astype(np.float64), quant_case.EXPECTED[prec])   # exact in FP32
    np.testing.assert_array_equal(got, np.repeat(want[None, :], n, axis=0))
    m.close()
