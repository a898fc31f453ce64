"""Host-side checks of the C ABI that need no device: blob parsing and argument validation.
Run against the product library by tests/test_abi_cpu.py, and against the host-sanitizer
build (AddressSanitizer + UndefinedBehaviorSanitizer) in a child process:
`python -m tests.abi_host_checks <library>`."""
import ctypes
import sys

import numpy as np

from paper_2512_13965_amd import inputs

OK, EINVAL, EUNSUPPORTED = 0, -1, -4
FP32, BF16, FP8 = 0, 1, 2


class Cond(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("log_tau", "c", "y_in", "sin_th", "log_aspect", "omega_x")]


class Exit(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("face", "pos", "dir_cos", "dir_sin", "path")]


def _create(L, blob, prec):
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    return L.gmc_model_create(buf, len(blob), prec, ctypes.byref(h))


def run(L):
    P, I64, U64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    L.gmc_last_error.restype = ctypes.c_char_p
    L.gmc_model_create.argtypes = [P, ctypes.c_size_t, I, ctypes.POINTER(P)]
    L.gmc_transmit.argtypes = [P, Cond, I64, I, U64, U64, P, P, Exit, P]
    L.mc_transmit.argtypes = [Cond, I64, I, U64, U64, Exit, P, P]
    L.gmc_decode.argtypes = [P, I64, Exit, P, P]
    L.gmc_uncollided_split.argtypes = [Cond, I64, U64, U64, P, Exit, P]
    L.gmc_world_set_streaming.argtypes = [P, I]
    L.gmc_world_transmissions.argtypes = [P, P]
    L.gmc_model_destroy.argtypes = [P]
    L.gmc_world_footprint.argtypes = [I64, ctypes.c_int32, I64, P]
    b = inputs.pack_blob(inputs.random_weights(256, 1))
    bad = bytearray(b)
    bad[0:8] = b"XXXXXXXX"
    assert _create(L, bad, FP32) == EINVAL
    assert b"magic" in L.gmc_last_error()
    assert _create(L, b[:-4], FP32) == EINVAL
    assert _create(L, b[:40], FP32) == EINVAL
    assert _create(L, b + b"\0\0\0\0", FP32) == EINVAL
    assert _create(L, b, 7) == EINVAL
    w = inputs.random_weights(256, 1)
    w.act_scale[2] = 0.3
    assert _create(L, inputs.pack_blob(w), FP8) == EINVAL
    # an FP8 layer's 2 w_scale act_scale must be an E8M0 value (2^-127 .. 2^127)
    w = inputs.random_weights(256, 1)
    w.act_scale[1], w.w_scale[1] = 2.0 ** -70, 2.0 ** -60
    assert _create(L, inputs.pack_blob(w), FP8) == EINVAL
    assert b"E8M0" in L.gmc_last_error()
    w = inputs.random_weights(256, 1)
    w.W[1][3, 4] = np.nan
    assert _create(L, inputs.pack_blob(w), FP32) == EINVAL
    # FP32 is built for H <= 256 only; H = 64 is built for no precision
    assert _create(L, inputs.pack_blob(inputs.random_weights(512, 1)), FP32) == EUNSUPPORTED
    assert _create(L, inputs.pack_blob(inputs.random_weights(64, 1)), BF16) == EUNSUPPORTED
    # blob flags: bit 0 XY geometry (11 inputs), bit 1 fitted on collided exits (boundary models),
    # bit 2 the residual network (a plain five-layer blob with it set does not parse)
    assert _create(L, inputs.pack_blob(inputs.random_weights(256, 1, flags=4)), FP32) == EINVAL
    assert _create(L, inputs.pack_blob(inputs.random_weights(256, 1, flags=8)), FP32) == EINVAL
    # the residual network: FP32 at H = 128 and BF16 only; 3 blocks of embedding width 32
    fw = inputs.random_film_weights(128, 1)
    fb = inputs.pack_blob(fw)
    assert _create(L, fb, FP8) == EUNSUPPORTED
    assert _create(L, inputs.pack_blob(inputs.random_film_weights(256, 1)), FP32) == EUNSUPPORTED
    assert _create(L, fb[:-4], BF16) == EINVAL
    assert _create(L, inputs.pack_blob(inputs.random_film_weights(128, 1, emb=64)), BF16) == EINVAL
    assert _create(L, inputs.pack_blob(inputs.random_film_weights(128, 1, blocks=2)), BF16) == EINVAL
    fw.W[4][2, 3] = np.inf
    assert _create(L, inputs.pack_blob(fw), BF16) == EINVAL
    assert _create(L, inputs.pack_blob(inputs.random_weights(256, 1, flags=1)), FP32) == EINVAL
    assert _create(L, inputs.pack_blob(inputs.random_weights(256, 1, n_in=inputs.N_IN_INTERNAL, flags=2)),
                   FP32) == EINVAL
    cond, out = Cond(), Exit()
    assert L.gmc_transmit(None, cond, 10, 16, 0, 0, None, None, out, None) == EINVAL
    assert L.mc_transmit(cond, 10, 5, 0, 0, out, None, None) == EINVAL
    assert L.mc_transmit(cond, -1, 0, 0, 0, out, None, None) == EINVAL
    assert L.mc_transmit(cond, 0, 0, 0, 0, out, None, None) == OK       # empty batch
    assert L.mc_transmit(cond, 10, 0, 0, 0, out, None, None) == EINVAL
    assert L.gmc_decode(None, 10, out, None, None) == EINVAL
    assert L.gmc_uncollided_split(cond, 10, 0, 0, None, out, None) == EINVAL
    assert L.gmc_uncollided_split(cond, -1, 0, 0, None, out, None) == EINVAL
    assert L.gmc_uncollided_split(cond, 0, 0, 0, None, out, None) == OK
    assert L.gmc_world_set_streaming(None, 4) == EINVAL
    assert L.gmc_world_transmissions(None, None) == EINVAL
    assert L.gmc_model_destroy(None) == EINVAL
    nbytes = ctypes.c_size_t()
    assert L.gmc_world_footprint(1 << 20, 4, 1 << 16, ctypes.byref(nbytes)) == OK and nbytes.value > 0
    assert L.gmc_world_footprint(0, 4, 1 << 16, ctypes.byref(nbytes)) == EINVAL


if __name__ == "__main__":
    run(ctypes.CDLL(sys.argv[1]))
    print("host checks passed")
