"""CPU checks of the C ABI: the library loads, exports every function include/gmc.h declares,
and rejects bad arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2512_13965_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                            text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def binding():
    from paper_2512_13965_amd import binding as b
    b.lib()
    return b


def test_header_compiles_as_c():
    for h in HEADERS:
        subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", h])


def test_every_declared_symbol_is_exported(binding):
    names = _declared_functions()
    assert "gmc_transmit" in names and "mc_transmit" in names
    out = subprocess.check_output(["nm", "-D", "--defined-only", binding.LIB_PATH], text=True)
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def _blob(H=256):
    return bytearray(inputs.pack_blob(inputs.random_weights(H, 1)))


def _create(binding, blob, prec):
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    return binding.lib().gmc_model_create(buf, len(blob), prec, ctypes.byref(h))


def test_model_create_rejects_bad_blobs(binding):
    L = binding.lib()
    b = _blob()
    bad = bytearray(b); bad[0:8] = b"XXXXXXXX"
    assert _create(binding, bad, binding.FP32) == binding.GMC_EINVAL
    assert b"magic" in L.gmc_last_error()
    assert _create(binding, b[:-4], binding.FP32) == binding.GMC_EINVAL
    assert _create(binding, b, 7) == binding.GMC_EINVAL
    w = inputs.random_weights(256, 1)
    w.act_scale[2] = 0.3
    assert _create(binding, inputs.pack_blob(w), binding.FP8_E4M3) == binding.GMC_EINVAL
    w = inputs.random_weights(256, 1)
    w.W[1][3, 4] = np.nan
    assert _create(binding, inputs.pack_blob(w), binding.FP32) == binding.GMC_EINVAL
    # FP32 is built for H <= 256 only; H = 64 is built for no precision
    assert _create(binding, _blob(512), binding.FP32) == binding.GMC_EUNSUPPORTED
    assert _create(binding, _blob(64), binding.BF16) == binding.GMC_EUNSUPPORTED
    # blob flags: bit 0 XY geometry (11 inputs), bit 1 fitted on collided exits (boundary models)
    assert _create(binding, inputs.pack_blob(inputs.random_weights(256, 1, flags=4)),
                   binding.FP32) == binding.GMC_EINVAL
    assert _create(binding, inputs.pack_blob(inputs.random_weights(256, 1, flags=1)),
                   binding.FP32) == binding.GMC_EINVAL
    assert _create(binding, inputs.pack_blob(inputs.random_weights(256, 1, n_in=inputs.N_IN_INTERNAL,
                                                                   flags=2)), binding.FP32) == binding.GMC_EINVAL


def test_sampling_calls_reject_bad_arguments_without_a_device(binding):
    L = binding.lib()
    cond = binding._Cond(None, None, None, None)
    out = binding._Exit(None, None, None, None, None)
    assert L.gmc_transmit(None, cond, 10, 16, 0, 0, None, None, out, None) == binding.GMC_EINVAL
    assert L.mc_transmit(cond, 10, 5, 0, 0, out, None, None) == binding.GMC_EINVAL
    assert L.mc_transmit(cond, -1, 0, 0, 0, out, None, None) == binding.GMC_EINVAL
    assert L.mc_transmit(cond, 0, 0, 0, 0, out, None, None) == binding.GMC_OK     # empty batch
    assert L.mc_transmit(cond, 10, 0, 0, 0, out, None, None) == binding.GMC_EINVAL
    assert L.gmc_decode(None, 10, out, None, None) == binding.GMC_EINVAL
    assert L.gmc_uncollided_split(cond, 10, 0, 0, None, out, None) == binding.GMC_EINVAL
    assert L.gmc_uncollided_split(cond, -1, 0, 0, None, out, None) == binding.GMC_EINVAL
    assert L.gmc_uncollided_split(cond, 0, 0, 0, None, out, None) == binding.GMC_OK
    L.gmc_world_set_streaming.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.gmc_world_transmissions.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert L.gmc_world_set_streaming(None, 4) == binding.GMC_EINVAL
    assert L.gmc_world_transmissions(None, None) == binding.GMC_EINVAL
    assert L.gmc_model_destroy(None) == binding.GMC_EINVAL
