"""Thin Python binding of libgmc.so (the C ABI in include/gmc.h).

Only argument marshalling lives here: torch provides device memory and streams, every step of
the sampling path runs in the library's HIP kernels.  Loading fails loudly if the library has
not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # noqa: F401  (must be loaded first: the library then shares torch's HIP runtime)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgmc.so")

GMC_OK, GMC_EINVAL, GMC_ENOMEM, GMC_EDEVICE, GMC_EUNSUPPORTED = 0, -1, -2, -3, -4
FP32, BF16, FP8_E4M3 = 0, 1, 2
MODE_CONTINUOUS, MODE_ANALOG = 0, 1
SAMPLER_GMC, SAMPLER_MC = 0, 1
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8_E4M3}


class GmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class _Cond(ctypes.Structure):
    _fields_ = [("log_tau", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("y_in", ctypes.c_void_p), ("sin_th", ctypes.c_void_p),
                ("log_aspect", ctypes.c_void_p), ("omega_x", ctypes.c_void_p)]


class _CondInternal(ctypes.Structure):
    _fields_ = [("log_tau", ctypes.c_void_p), ("c", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("cos_phi", ctypes.c_void_p), ("sin_phi", ctypes.c_void_p)]


class _Exit(ctypes.Structure):
    _fields_ = [("face", ctypes.c_void_p), ("pos", ctypes.c_void_p),
                ("dir_cos", ctypes.c_void_p), ("dir_sin", ctypes.c_void_p),
                ("path", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, U64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        L.gmc_last_error.restype = ctypes.c_char_p
        L.gmc_model_create.argtypes = [P, ctypes.c_size_t, I, ctypes.POINTER(P)]
        L.gmc_model_destroy.argtypes = [P]
        L.gmc_model_info.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I)]
        L.gmc_transmit.argtypes = [P, _Cond, I64, I, U64, U64, P, P, _Exit, P]
        L.gmc_sample.argtypes = [P, _Cond, I64, I, I, U64, U64, P, P, _Exit, P]
        L.mc_transmit.argtypes = [_Cond, I64, I, U64, U64, _Exit, P, P]
        L.gmc_decode.argtypes = [P, I64, _Exit, P, P]
        L.gmc_model_inputs.argtypes = [P, ctypes.POINTER(I)]
        L.gmc_sample_internal.argtypes = [P, _CondInternal, I64, I, I, U64, U64, P, P, _Exit, P]
        L.mc_transmit_internal.argtypes = [_CondInternal, I64, I, U64, U64, _Exit, P, P]
        L.gmc_uncollided_split.argtypes = [_Cond, I64, U64, U64, P, _Exit, P]
        L.gmc_device_init.argtypes = []
        for name in ("gmc_model_create", "gmc_model_destroy", "gmc_model_info", "gmc_transmit",
                     "mc_transmit", "gmc_decode", "gmc_sample", "gmc_model_inputs",
                     "gmc_sample_internal", "mc_transmit_internal", "gmc_uncollided_split", "gmc_device_init"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


_ready_devices = set()


def device_init():
    """gmc_device_init on the current device (once per device): the analog walk's counters."""
    dev = torch.cuda.current_device()
    if dev not in _ready_devices:
        _check(lib().gmc_device_init())
        _ready_devices.add(dev)


def _check(rc: int):
    if rc != GMC_OK:
        raise GmcError(rc, lib().gmc_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, n, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() >= n):
        raise ValueError(f"{name}: expected a contiguous {dtype} device tensor of >= {n} elements")


@dataclass
class DeviceCond:
    """Device SoA of entry conditions (float32 tensors of equal length); log_aspect is
    optional (rectangular cells)."""
    log_tau: torch.Tensor
    c: torch.Tensor
    y_in: torch.Tensor
    sin_th: torch.Tensor
    log_aspect: torch.Tensor | None = None
    omega_x: torch.Tensor | None = None

    @classmethod
    def from_host(cls, cond, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        la = getattr(cond, "log_aspect", None)
        ox = getattr(cond, "omega_x", None)
        return cls(f(cond.log_tau), f(cond.c), f(cond.y_in), f(cond.sin_th),
                   None if la is None else f(la), None if ox is None else f(ox))

    def __len__(self):
        return int(self.log_tau.numel())

    def c_struct(self) -> _Cond:
        n = len(self)
        for nm in ("log_tau", "c", "y_in", "sin_th"):
            _need(getattr(self, nm), torch.float32, n, nm)
        for nm in ("log_aspect", "omega_x"):
            if getattr(self, nm) is not None:
                _need(getattr(self, nm), torch.float32, n, nm)
        return _Cond(self.log_tau.data_ptr(), self.c.data_ptr(), self.y_in.data_ptr(),
                     self.sin_th.data_ptr(),
                     None if self.log_aspect is None else self.log_aspect.data_ptr(),
                     None if self.omega_x is None else self.omega_x.data_ptr())


@dataclass
class DeviceCondInternal:
    """Device SoA of internal-model birth conditions (float32 tensors of equal length)."""
    log_tau: torch.Tensor
    c: torch.Tensor
    x: torch.Tensor
    y: torch.Tensor
    cos_phi: torch.Tensor
    sin_phi: torch.Tensor

    @classmethod
    def from_host(cls, cond, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        return cls(f(cond.log_tau), f(cond.c), f(cond.x), f(cond.y), f(cond.cos_phi), f(cond.sin_phi))

    def __len__(self):
        return int(self.log_tau.numel())

    def c_struct(self) -> _CondInternal:
        n = len(self)
        names = ("log_tau", "c", "x", "y", "cos_phi", "sin_phi")
        for nm in names:
            _need(getattr(self, nm), torch.float32, n, nm)
        return _CondInternal(*(getattr(self, nm).data_ptr() for nm in names))


@dataclass
class DeviceExit:
    face: torch.Tensor
    pos: torch.Tensor
    dir_cos: torch.Tensor
    dir_sin: torch.Tensor
    path: torch.Tensor

    @classmethod
    def empty(cls, n: int, device="cuda"):
        e = lambda dt: torch.empty(n, dtype=dt, device=device)
        return cls(e(torch.int32), e(torch.float32), e(torch.float32), e(torch.float32),
                   e(torch.float32))

    def c_struct(self, n: int) -> _Exit:
        _need(self.face, torch.int32, n, "face")
        for nm in ("pos", "dir_cos", "dir_sin", "path"):
            _need(getattr(self, nm), torch.float32, n, nm)
        return _Exit(self.face.data_ptr(), self.pos.data_ptr(), self.dir_cos.data_ptr(),
                     self.dir_sin.data_ptr(), self.path.data_ptr())

    def to_host(self) -> dict:
        return {k: getattr(self, k).cpu().numpy() for k in ("face", "pos", "dir_cos", "dir_sin", "path")}


class Model:
    """Device copy of a velocity network (gmc_model_create / gmc_model_destroy)."""

    def __init__(self, blob: bytes, precision):
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().gmc_model_create(buf, len(blob), int(precision), ctypes.byref(h)))
        self._h = h
        hid, prec = ctypes.c_int(), ctypes.c_int()
        _check(lib().gmc_model_info(h, ctypes.byref(hid), ctypes.byref(prec)))
        self.hidden, self.precision = hid.value, prec.value
        nin = ctypes.c_int()
        _check(lib().gmc_model_inputs(h, ctypes.byref(nin)))
        self.n_in = nin.value          # 10: boundary model, 12: internal model

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _check(lib().gmc_model_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gmc_transmit(model: Model, cond: DeviceCond, K: int, seed: int, id_base: int = 0,
                 noise: torch.Tensor | None = None, raw: torch.Tensor | None = None,
                 out: DeviceExit | None = None, n: int | None = None, stream=None) -> DeviceExit:
    n = len(cond) if n is None else n
    if out is None:
        out = DeviceExit.empty(n, cond.log_tau.device)
    if noise is not None:
        _need(noise, torch.float32, 5 * n, "noise")
    if raw is not None:
        _need(raw, torch.float32, 5 * n, "raw")
    _check(lib().gmc_transmit(model.handle, cond.c_struct(), n, int(K), seed, id_base,
                              _ptr(noise), _ptr(raw), out.c_struct(n), _stream(stream)))
    return out


INTEGRATORS = {"euler": 0, "rk4": 1}


def gmc_sample(model: Model, cond: DeviceCond, integrator: str, K: int, seed: int,
               id_base: int = 0, noise: torch.Tensor | None = None,
               raw: torch.Tensor | None = None, out: DeviceExit | None = None,
               n: int | None = None, stream=None) -> DeviceExit:
    """gmc_sample: the generative sampler with integrator "euler" or "rk4" over K steps."""
    n = len(cond) if n is None else n
    if integrator not in INTEGRATORS:
        raise ValueError(f"integrator must be one of {sorted(INTEGRATORS)}")
    if out is None:
        out = DeviceExit.empty(n, cond.log_tau.device)
    if noise is not None:
        _need(noise, torch.float32, 5 * n, "noise")
    if raw is not None:
        _need(raw, torch.float32, 5 * n, "raw")
    _check(lib().gmc_sample(model.handle, cond.c_struct(), n, INTEGRATORS[integrator], int(K),
                            seed, id_base, _ptr(noise), _ptr(raw), out.c_struct(n),
                            _stream(stream)))
    return out


def gmc_sample_internal(model: Model, cond: DeviceCondInternal, integrator: str, K: int, seed: int,
                        id_base: int = 0, noise: torch.Tensor | None = None,
                        raw: torch.Tensor | None = None, out: DeviceExit | None = None,
                        n: int | None = None, stream=None) -> DeviceExit:
    """gmc_sample_internal: the internal (volumetric-source) model's sampler."""
    n = len(cond) if n is None else n
    if integrator not in INTEGRATORS:
        raise ValueError(f"integrator must be one of {sorted(INTEGRATORS)}")
    if out is None:
        out = DeviceExit.empty(n, cond.log_tau.device)
    if noise is not None:
        _need(noise, torch.float32, 5 * n, "noise")
    if raw is not None:
        _need(raw, torch.float32, 5 * n, "raw")
    _check(lib().gmc_sample_internal(model.handle, cond.c_struct(), n, INTEGRATORS[integrator], int(K),
                                     seed, id_base, _ptr(noise), _ptr(raw), out.c_struct(n),
                                     _stream(stream)))
    return out


def mc_transmit_internal(cond: DeviceCondInternal, mode: int, seed: int, id_base: int = 0,
                         ncoll: torch.Tensor | None = None, out: DeviceExit | None = None,
                         n: int | None = None, stream=None) -> DeviceExit:
    """mc_transmit_internal: the analog walk from a birth point inside the cell."""
    n = len(cond) if n is None else n
    if out is None:
        out = DeviceExit.empty(n, cond.log_tau.device)
    if ncoll is not None:
        _need(ncoll, torch.int32, n, "ncoll")
    device_init()
    _check(lib().mc_transmit_internal(cond.c_struct(), n, int(mode), seed, id_base, out.c_struct(n),
                                      _ptr(ncoll), _stream(stream)))
    return out


def mc_transmit(cond: DeviceCond, mode: int, seed: int, id_base: int = 0,
                ncoll: torch.Tensor | None = None, out: DeviceExit | None = None,
                n: int | None = None, stream=None) -> DeviceExit:
    n = len(cond) if n is None else n
    if out is None:
        out = DeviceExit.empty(n, cond.log_tau.device)
    if ncoll is not None:
        _need(ncoll, torch.int32, n, "ncoll")
    device_init()
    _check(lib().mc_transmit(cond.c_struct(), n, int(mode), seed, id_base, out.c_struct(n),
                             _ptr(ncoll), _stream(stream)))
    return out


def uncollided_split(cond: DeviceCond, seed: int, id_base: int = 0, flag: torch.Tensor | None = None,
                     out: DeviceExit | None = None, n: int | None = None, stream=None):
    """gmc_uncollided_split: flag[i] = 1 where particle i crosses its cell without a collision,
    with its exit written to out[i].  Returns (flag, out)."""
    n = len(cond) if n is None else n
    if out is None:
        out = DeviceExit.empty(n, cond.log_tau.device)
    if flag is None:
        flag = torch.zeros(n, dtype=torch.int32, device=cond.log_tau.device)
    _need(flag, torch.int32, n, "flag")
    _check(lib().gmc_uncollided_split(cond.c_struct(), n, seed, id_base, _ptr(flag), out.c_struct(n),
                                      _stream(stream)))
    return flag, out


def gmc_decode(raw: torch.Tensor, n: int, out: DeviceExit | None = None,
               flags: torch.Tensor | None = None, stream=None) -> DeviceExit:
    _need(raw, torch.float32, 5 * n, "raw")
    if out is None:
        out = DeviceExit.empty(n, raw.device)
    if flags is not None:
        _need(flags, torch.int32, n, "flags")
    _check(lib().gmc_decode(_ptr(raw), n, out.c_struct(n), _ptr(flags), _stream(stream)))
    return out


# ------------------------------------------------------------------------------------------
# transport world (gmc_world_* / gmc_problem_* / gmc_transport_step)
# ------------------------------------------------------------------------------------------

class _ProblemDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("L", ctypes.c_double),
                ("tau", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("src_x0", ctypes.c_int32), ("src_y0", ctypes.c_int32),
                ("src_nx", ctypes.c_int32), ("src_ny", ctypes.c_int32),
                ("reflect", ctypes.c_int32), ("w_min", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("src_face", ctypes.c_int32), ("Ly", ctypes.c_double), ("xy", ctypes.c_int32),
                ("max_visits", ctypes.c_int64)]


def _transport_sigs(L):
    P, I32, I64, U64, I = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    L.gmc_world_footprint.argtypes = [I64, I32, I64, ctypes.POINTER(ctypes.c_size_t)]
    L.gmc_world_create.argtypes = [I64, I32, I64, ctypes.POINTER(P)]
    L.gmc_world_destroy.argtypes = [P]
    L.gmc_problem_add.argtypes = [P, ctypes.POINTER(_ProblemDesc), ctypes.POINTER(I32), P]
    L.gmc_problem_remove.argtypes = [P, I32]
    L.gmc_world_inject.argtypes = [P, I32, U64, I64, P, ctypes.POINTER(I64)]
    L.gmc_transport_step.argtypes = [P, I, P, I, P, ctypes.POINTER(I64)]
    L.gmc_problem_alive.argtypes = [P, I32, ctypes.POINTER(I64)]
    L.gmc_problem_tally.argtypes = [P, I32, P, P, P, P, P]
    L.gmc_problem_path_tally.argtypes = [P, I32, P, P, P, P, P, P]
    L.gmc_world_set_integrator.argtypes = [P, I]
    L.gmc_world_set_graphs.argtypes = [P, I]
    L.gmc_world_set_streaming.argtypes = [P, I]
    L.gmc_world_transmissions.argtypes = [P, ctypes.POINTER(I64)]
    L.gmc_world_set_source_model.argtypes = [P, P, I]
    for name in ("gmc_world_set_integrator", "gmc_world_set_graphs", "gmc_world_set_source_model", "gmc_world_footprint", "gmc_world_create", "gmc_world_destroy", "gmc_problem_add",
                 "gmc_problem_remove", "gmc_world_inject", "gmc_transport_step",
                 "gmc_problem_alive", "gmc_problem_tally", "gmc_problem_path_tally"):
        getattr(L, name).restype = ctypes.c_int


def world_footprint(capacity: int, max_problems: int, max_cells: int) -> int:
    L = lib()
    _transport_sigs(L)
    b = ctypes.c_size_t()
    _check(L.gmc_world_footprint(capacity, max_problems, max_cells, ctypes.byref(b)))
    return int(b.value)


class World:
    """Device particle bank + problem slots (gmc_world_create / gmc_world_destroy)."""

    def __init__(self, capacity: int, max_problems: int = 1, max_cells: int = 1 << 16):
        self._L = lib()
        _transport_sigs(self._L)
        h = ctypes.c_void_p()
        _check(self._L.gmc_world_create(capacity, max_problems, max_cells, ctypes.byref(h)))
        self._h = h
        self.capacity = capacity
        self._shapes = {}

    def add_problem(self, problem, seed: int, stream=None) -> int:
        import numpy as np
        tau = np.ascontiguousarray(problem.tau, np.float64)
        c = np.ascontiguousarray(problem.c, np.float64)
        d = _ProblemDesc(problem.nx, problem.ny, problem.L, tau.ctypes.data, c.ctypes.data,
                         problem.src_x0, problem.src_y0, problem.src_nx, problem.src_ny,
                         int(problem.reflect), problem.w_min, seed, int(getattr(problem, "src_face", -1)),
                         float(getattr(problem, "Ly", 0.0)), int(bool(getattr(problem, "xy", False))),
                         int(getattr(problem, "max_visits", 0)))
        pid = ctypes.c_int32()
        _check(self._L.gmc_problem_add(self._h, ctypes.byref(d), ctypes.byref(pid), _stream(stream)))
        self._shapes[pid.value] = problem.n_cells
        return pid.value

    def remove(self, pid: int):
        _check(self._L.gmc_problem_remove(self._h, pid))
        self._shapes.pop(pid, None)

    def inject(self, pid: int, h_begin: int, count: int, stream=None) -> int:
        n = ctypes.c_int64()
        _check(self._L.gmc_world_inject(self._h, pid, h_begin, count, _stream(stream), ctypes.byref(n)))
        return n.value

    def set_integrator(self, integrator: str):
        """ODE integrator ("euler" or "rk4") of later generative-sampler steps."""
        if integrator not in INTEGRATORS:
            raise ValueError(f"integrator must be one of {sorted(INTEGRATORS)}")
        _check(self._L.gmc_world_set_integrator(self._h, INTEGRATORS[integrator]))

    def set_source_model(self, model: Model | None, K: int = 16):
        """Births sampled by an internal model (None: analog first leg)."""
        _check(self._L.gmc_world_set_source_model(self._h, None if model is None else model.handle, int(K)))

    def set_streaming(self, max_crossings: int):
        _check(self._L.gmc_world_set_streaming(self._h, int(max_crossings)))

    def transmissions(self) -> int:
        v = ctypes.c_int64()
        _check(self._L.gmc_world_transmissions(self._h, ctypes.byref(v)))
        return v.value

    def set_graphs(self, enable: bool = True):
        """Replay captured HIP graphs of the transport step per particle-count bucket."""
        _check(self._L.gmc_world_set_graphs(self._h, 1 if enable else 0))

    def step(self, sampler: int, model: Model | None = None, K: int = 16, stream=None) -> int:
        n = ctypes.c_int64()
        _check(self._L.gmc_transport_step(self._h, sampler, None if model is None else model.handle,
                                          K, _stream(stream), ctypes.byref(n)))
        return n.value

    def alive(self, pid: int) -> int:
        n = ctypes.c_int64()
        _check(self._L.gmc_problem_alive(self._h, pid, ctypes.byref(n)))
        return n.value

    def tally(self, pid: int, stream=None) -> dict:
        """Per-cell FP64 tallies summed over the histories so far: flux, absorbed, leak, cutoff
        (gmc_problem_tally) and the path tallies wpath, path, visits, rejected_w, rejected_n
        (gmc_problem_path_tally)."""
        import numpy as np
        m = self._shapes[pid]
        out = {k: np.zeros(m) for k in ("flux", "absorbed", "leak", "cutoff", "wpath", "path", "visits",
                                        "rejected_w", "rejected_n")}
        _check(self._L.gmc_problem_tally(self._h, pid, out["flux"].ctypes.data,
                                         out["absorbed"].ctypes.data, out["leak"].ctypes.data,
                                         out["cutoff"].ctypes.data, _stream(stream)))
        _check(self._L.gmc_problem_path_tally(self._h, pid, out["wpath"].ctypes.data, out["path"].ctypes.data,
                                              out["visits"].ctypes.data, out["rejected_w"].ctypes.data,
                                              out["rejected_n"].ctypes.data, _stream(stream)))
        return out

    def close(self):
        if self._h:
            _check(self._L.gmc_world_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
