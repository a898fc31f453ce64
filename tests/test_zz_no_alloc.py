"""mc_transmit_noalloc (the allocation-free analog walk) through the C ABI against mc_transmit:
the same walks bit for bit, on two calls in a row, the second with fewer particles (its
counter array keeps the first call's contents, so the call must clear what it uses)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2512_13965_amd import inputs
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _walk(binding, fn_name, cond, n, mode, seed, id_base):
    L = binding.lib()
    fn = getattr(L, fn_name)
    fn.argtypes = [binding._Cond, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, binding._Exit,
                   ctypes.c_void_p, ctypes.c_void_p]
    fn.restype = ctypes.c_int
    out = binding.DeviceExit.empty(n)
    ncoll = torch.zeros(n, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(cond.c_struct(), n, mode, seed, id_base, out.c_struct(n), ctypes.c_void_p(ncoll.data_ptr()), stream)
    assert rc == binding.GMC_OK, L.gmc_last_error()
    torch.cuda.synchronize()
    res = out.to_host()
    res["ncoll"] = ncoll.cpu().numpy()
    return res


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_walk_matches_mc_transmit(mode):
    binding = require_gpu()
    L = binding.lib()
    assert L.gmc_device_init() == binding.GMC_OK
    for n, tau, seed, id_base in ((300_000, 20.0, 7, 0), (12_345, 3.0, 8, 1 << 33)):
        c = inputs.transmission_conditions(n, seed, log_tau_range=(np.log(0.5), np.log(tau)))
        cond = binding.DeviceCond.from_host(c)
        want = _walk(binding, "mc_transmit", cond, n, mode, seed, id_base)
        got = _walk(binding, "mc_transmit_noalloc", cond, n, mode, seed, id_base)
        for k in want:
            np.testing.assert_array_equal(got[k], want[k], err_msg=f"{k} (n = {n})")
        assert (want["face"] >= (-1 if mode == 1 else 0)).all()
    # sizes beyond the counter's range are refused before any device work
    empty = binding._Cond(None, None, None, None)
    none = binding._Exit(None, None, None, None, None)
    assert L.mc_transmit_noalloc(empty, (1 << 62) + 1, 0, 0, 0, none, None, None) == binding.GMC_EINVAL
