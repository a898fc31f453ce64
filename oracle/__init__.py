"""CPU oracle for Generative Monte Carlo cell transmission -- TEST INFRASTRUCTURE ONLY.

Only the tests, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py` may import
this package.  It shares no code with the GPU path (`paper_2512_13965_amd`); the only
module both sides use is the seeded input generator `paper_2512_13965_amd.inputs`, which
holds none of the method's arithmetic.

Contents
  * `gmc_oracle.c` (built to `liboracle.so`): Philox4x32-10, Box-Muller noise, the analog
    walk through one cell in FP64 (modes C and A), and FP64 cell-to-cell transport.
  * this module: ctypes bindings for the above, and the FP64 velocity-MLP sampler (explicit
    Euler and classic RK4) with optional BF16 / FP8-e4m3 quantisation emulation, the residual
    network with adaptive modulation (FP64 or BF16 operands), plus the exit decoder.

Paper references are to arXiv 2512.13965 (sections and equation numbers in order of
appearance).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "gmc_oracle.c")

FACE_ABSORBED = -1
FACE_CAPPED = -2


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, IEEE semantics, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp,
                               SRC_PATH, "-lm", "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_u01.argtypes = [ctypes.c_uint32]
        L.orc_u01.restype = ctypes.c_double
        L.orc_noise_batch.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P]
        L.orc_mc_transmit.argtypes = [P, P, P, P, P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.c_uint64, P, P, P, P, P, P, ctypes.c_int]
        L.orc_mc_transmit_internal.argtypes = [P, P, P, P, P, P, ctypes.c_int64, ctypes.c_int,
                                               ctypes.c_uint64, ctypes.c_uint64, P, P, P, P, P, P,
                                               ctypes.c_int]
        L.orc_uncollided_split.argtypes = [P, P, P, P, P, P, ctypes.c_int64, ctypes.c_uint64,
                                           ctypes.c_uint64, P, P, P, P, P, P]
        L.orc_transport.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, P, P,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, P, P, P, ctypes.c_int,
                                    ctypes.c_uint32, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------------------
# random numbers
# ----------------------------------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def u01(u: int) -> float:
    return float(lib().orc_u01(ctypes.c_uint32(int(u) & 0xFFFFFFFF)))


def noise(seed: int, id_base: int, n: int) -> np.ndarray:
    """z ~ N(0, I_5) per sample from Philox + Box-Muller, FP64, layout [5][n]."""
    z = np.zeros((5, n), np.float64)
    lib().orc_noise_batch(seed, id_base, n, _p(z))
    return z


# ----------------------------------------------------------------------------------------
# analog walk (paper section "Monte Carlo Method", eq. 4; modes C = implicit capture, A)
# ----------------------------------------------------------------------------------------

def mc_transmit(cond, mode: int, seed: int, id_base: int = 0, nthreads: int = 1) -> dict:
    """FP64 analog transmissions of a canonical batch.  mode 0 = C (continuous absorption,
    flights from sigma_s = c*tau), 1 = A (analog absorption); rectangular cells [0, A] x [0, 1]
    when cond.log_aspect is given.  Returns numpy arrays: face (int32; -1 absorbed), pos (a
    fraction of the exit face), u, v, len (float64, units of the entry face), ncoll (uint32)."""
    n = len(cond)
    lt = np.ascontiguousarray(cond.log_tau, np.float32)
    cc = np.ascontiguousarray(cond.c, np.float32)
    yy = np.ascontiguousarray(cond.y_in, np.float32)
    ss = np.ascontiguousarray(cond.sin_th, np.float32)
    la = getattr(cond, "log_aspect", None)
    la = None if la is None else np.ascontiguousarray(la, np.float32)
    ox = getattr(cond, "omega_x", None)
    ox = None if ox is None else np.ascontiguousarray(ox, np.float32)
    out = dict(face=np.zeros(n, np.int32), pos=np.zeros(n), u=np.zeros(n), v=np.zeros(n),
               len=np.zeros(n), ncoll=np.zeros(n, np.uint32))
    lib().orc_mc_transmit(_p(lt), _p(cc), _p(yy), _p(ss), None if la is None else _p(la),
                          None if ox is None else _p(ox), n, mode, seed, id_base,
                          _p(out["face"]), _p(out["pos"]), _p(out["u"]), _p(out["v"]),
                          _p(out["len"]), _p(out["ncoll"]), nthreads)
    return out


def uncollided_split(cond, seed: int, id_base: int = 0) -> dict:
    """First-flight split (an analytic variant beside the paper's single model): flag = 1 where
    the particle crosses without a collision (probability exp(-c tau d_b) against Philox word 0
    of counter (id, 0, 4)); face, pos, u, v, len of the entry ray's exit for every particle."""
    n = len(cond)
    f32 = lambda a: None if a is None else np.ascontiguousarray(a, np.float32)
    arrs = [f32(cond.log_tau), f32(cond.c), f32(cond.y_in), f32(cond.sin_th),
            f32(getattr(cond, "log_aspect", None)), f32(getattr(cond, "omega_x", None))]
    out = dict(flag=np.zeros(n, np.int32), face=np.zeros(n, np.int32), pos=np.zeros(n), u=np.zeros(n),
               v=np.zeros(n), len=np.zeros(n))
    lib().orc_uncollided_split(*[None if a is None else _p(a) for a in arrs], n, seed, id_base,
                               _p(out["flag"]), _p(out["face"]), _p(out["pos"]), _p(out["u"]),
                               _p(out["v"]), _p(out["len"]))
    return out


def mc_transmit_internal(cond, mode: int, seed: int, id_base: int = 0, nthreads: int = 1) -> dict:
    """FP64 analog walks started inside the cell: particle i born at (x, y) with direction
    (cos_phi, sin_phi) in the cell's own frame.  Same modes and outputs as mc_transmit."""
    n = len(cond)
    arr = [np.ascontiguousarray(a, np.float32) for a in (cond.log_tau, cond.c, cond.x, cond.y,
                                                          cond.cos_phi, cond.sin_phi)]
    out = dict(face=np.zeros(n, np.int32), pos=np.zeros(n), u=np.zeros(n), v=np.zeros(n),
               len=np.zeros(n), ncoll=np.zeros(n, np.uint32))
    lib().orc_mc_transmit_internal(*(_p(a) for a in arr), n, mode, seed, id_base,
                                   _p(out["face"]), _p(out["pos"]), _p(out["u"]), _p(out["v"]),
                                   _p(out["len"]), _p(out["ncoll"]), nthreads)
    return out


def transport(problem, seed: int, h_begin: int, h_end: int, nthreads: int = 1) -> dict:
    """FP64 cell-to-cell transport (analog mode-C walk in every cell, track-length tally).
    A history still alive on reaching cell visit number problem.max_visits (0: 2^24; visit 0 is
    a volumetric birth's cell, 1 a surface birth's) ends there with its weight as cutoff.
    Returns sums over the histories: flux[n_cells], absorbed[n_cells], leak, cutoff, events, and
    the path tallies wpath (w_in * l), path (l) and visits [n_cells] (track length of every cell
    visit, "Transport Algorithm" third stage)."""
    tau = np.ascontiguousarray(problem.tau, np.float64)
    c = np.ascontiguousarray(problem.c, np.float64)
    flux = np.zeros(problem.n_cells)
    absorbed = np.zeros(problem.n_cells)
    sc = np.zeros(3)
    pt = np.zeros((3, problem.n_cells))
    lib().orc_transport(problem.nx, problem.ny, problem.L, float(getattr(problem, "Ly", 0.0)),
                        _p(tau), _p(c), problem.src_x0,
                        problem.src_y0, problem.src_nx, problem.src_ny, int(problem.reflect),
                        int(getattr(problem, "src_face", -1)), int(getattr(problem, "xy", False)),
                        problem.w_min, seed, h_begin, h_end,
                        _p(flux), _p(absorbed), _p(sc), nthreads, int(getattr(problem, "max_visits", 0)), _p(pt))
    return dict(flux=flux, absorbed=absorbed, leak=sc[0], cutoff=sc[1], events=sc[2], wpath=pt[0], path=pt[1],
                visits=pt[2])


# ----------------------------------------------------------------------------------------
# quantisation emulation (BF16 and OCP FP8 e4m3, round-to-nearest-even)
# ----------------------------------------------------------------------------------------

def round_bf16(a) -> np.ndarray:
    """Round each value to the nearest bfloat16 (8 significant bits, ties to even), FP64 out.
    Values are first taken to float32 (the kernel holds them in float32)."""
    f = np.asarray(a, np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def round_e4m3(a) -> np.ndarray:
    """Round to the nearest OCP FP8 e4m3 value (bias 7, 3 mantissa bits, subnormals down to
    2^-9, largest finite 448), ties to even, saturating at +-448.  FP64 in and out."""
    x = np.asarray(a, np.float64)
    s = np.sign(x)
    m = np.abs(x)
    m = np.minimum(m, 448.0)
    # exponent e of the binade [2^e, 2^(e+1)) holding m, clamped below at -6 so that the
    # subnormal range keeps the spacing 2^-9
    _, ex = np.frexp(np.where(m > 0, m, 1.0))
    e = np.maximum(ex.astype(np.float64) - 1.0, -6.0)
    q = 2.0 ** (e - 3.0)                    # spacing of representable values in this binade
    r = np.round(m / q) * q                 # numpy rounds halves to even
    r = np.minimum(r, 448.0)
    return s * r


# ----------------------------------------------------------------------------------------
# velocity MLP + Euler sampler (paper "Conditional Flow Matching", eq. 8)
# ----------------------------------------------------------------------------------------

PREC_FP64 = "fp64"    # exact arithmetic of the network, no rounding
PREC_BF16 = "bf16"    # inputs of every layer and all weights rounded to bfloat16
PREC_FP8 = "fp8"      # hidden H x H layers in e4m3 with per-layer scales, first/last in bf16
# BF16 operands with the hidden activations carried scaled by -log2(e) (fold_exp2): the order
# in which the library's BF16 sampler evaluates the network
PREC_BF16_EXP2 = "bf16-exp2"
# PREC_FP8's roundings applied to the network of fold_exp2, with the activations that enter an
# e4m3 layer carried at half that factor (velocity_fp8_exp2): the order of the FP8 sampler
PREC_FP8_EXP2 = "fp8-exp2"

# -log2(e) and -ln 2 as float32 values
NEG_LOG2E_F32 = np.float32(-1.0 / math.log(2.0))
NEG_LN2_F32 = np.float32(-math.log(2.0))


def silu(a):
    with np.errstate(over="ignore"):       # exp(-a) -> inf for a << 0 gives the limit -0
        return a / (1.0 + np.exp(-a))


def condition_features(cond) -> np.ndarray:
    """Condition part of the network input.  Boundary model (entry conditions):
    (ln tau, c, 2*y_in - 1, sin theta_in), [n, 4], and for rectangular cells (conditions with a
    log_aspect) ln A as a fifth column, [n, 5]; in XY geometry (conditions with omega_x, sin_th
    being the in-plane y component) omega_x as the fifth column.  Internal model (birth conditions, which carry
    the birth position x, y and direction): (ln tau, c, 2x - 1, 2y - 1, cos phi, sin phi), [n, 6]."""
    f = lambda a: np.asarray(a, np.float64)
    if hasattr(cond, "x"):
        return np.stack([f(cond.log_tau), f(cond.c), 2.0 * f(cond.x) - 1.0, 2.0 * f(cond.y) - 1.0,
                         f(cond.cos_phi), f(cond.sin_phi)], axis=1)
    cols = [f(cond.log_tau), f(cond.c), 2.0 * f(cond.y_in) - 1.0, f(cond.sin_th)]
    if getattr(cond, "log_aspect", None) is not None:
        cols.append(f(cond.log_aspect))
    elif getattr(cond, "omega_x", None) is not None:       # XY geometry: omega_x
        cols.append(f(cond.omega_x))
    return np.stack(cols, axis=1)


def layer_affine(weights, l: int, h, precision=PREC_FP64):
    """Affine part W_l h + b_l of layer l (0-based) of the velocity network for a batch
    h [n, in] -> [n, out], with the operand rounding of `precision` (paper "Conditional Flow
    Matching", eq. 8, evaluated in reduced precision; the reading of the quantised network):
      * PREC_FP64: no rounding.
      * PREC_BF16: the layer input h and the weights W_l are rounded to bfloat16 (to nearest,
        ties to even); the products are summed exactly (FP64 here, FP32 on the matrix core);
        the bias b_l is added unrounded (its float32 value).
      * PREC_FP8: the hidden H x H layers (0 < l < last) take e4m3 operands: h divided by the
        layer's activation scale sa and W_l by its weight scale sw (both powers of two), each
        rounded to e4m3 (to nearest, ties to even, saturating at +-448); the exact sum of the
        products is multiplied by sa * sw and the unrounded bias added.  The first and the last
        layer are BF16 as above."""
    W = weights.W[l].astype(np.float64)
    b = weights.b[l].astype(np.float64)
    last = len(weights.W) - 1
    if precision == PREC_BF16 or (precision == PREC_FP8 and not 0 < l < last):
        return round_bf16(h) @ round_bf16(W).T + b
    if precision == PREC_FP8:
        sa = float(weights.act_scale[l])
        sw = float(weights.w_scale[l])
        return (round_e4m3(h / sa) @ round_e4m3(W / sw).T) * (sa * sw) + b
    return h @ W.T + b


def time_features(t) -> np.ndarray:
    """Time input of the residual network (its learned time embedding starts from these):
    sin and cos of pi 2^j t for j = 0, 1, 2, 3, as [sin pi t, cos pi t, sin 2 pi t, ...].  The
    lowest frequency makes t = 0 and t = 1 distinct."""
    out = []
    for j in range(4):
        a = math.pi * (2.0 ** j) * float(t)
        out += [math.sin(a), math.cos(a)]
    return np.array(out)


def film_velocity(weights, x, t, condf, precision=PREC_FP64):
    """v_theta(x, t | c) of the residual network with adaptive modulation (paper "Network
    Architecture and Inputs": learned embeddings of t and c, residual blocks modulated by the
    physical context; the layer details are this library's reading).  With phi = time_features(t)
    and u = [x, phi, c]:
        h_0 = W_in u + b_in
        e   = SiLU(W_e [phi, c] + b_e)                       (the embedding, width E)
        for each block j:  h_j = h_{j-1} + SiLU((1 + G_j e + g_j) * (A_j h_{j-1} + a_j)
                                                  + (S_j e + s_j))
        v   = W_o h_B + b_o
    PREC_BF16: every layer's input and weights rounded to bfloat16 (layer_affine's reading),
    and the residual stream h_j stored in bfloat16 (rounded after each block's sum)."""
    if precision not in (PREC_FP64, PREC_BF16):
        raise ValueError("the residual network is evaluated in FP64 or with BF16 operands")
    rd = round_bf16 if precision == PREC_BF16 else (lambda a: np.asarray(a, np.float64))
    W = [w.astype(np.float64) for w in weights.W]
    b = [v.astype(np.float64) for v in weights.b]
    lin = lambda l, a: rd(a) @ rd(W[l]).T + b[l]
    n = x.shape[0]
    phi = np.broadcast_to(time_features(t), (n, 8))
    h = rd(lin(0, np.concatenate([x, phi, condf], axis=1)))
    e = silu(lin(1, np.concatenate([phi, condf], axis=1)))
    nb = (len(W) - 3) // 3
    for j in range(nb):
        a = lin(2 + 3 * j, h)
        scale = 1.0 + lin(3 + 3 * j, e)
        shift = lin(4 + 3 * j, e)
        h = rd(h + silu(scale * a + shift))
    return lin(2 + 3 * nb, h)


def fold_exp2(weights):
    """The same network with every hidden activation carried scaled by -log2(e): the first
    layer's weights and every hidden bias multiplied by -log2(e), the output layer's weights by
    -ln 2, each product rounded to float32.  A layer then computes a' = -log2(e) a, and its
    scaled activation -log2(e) SiLU(a) is a' / (1 + 2^a'); the next layer's inputs carry the
    factor, which the following layer's unscaled weights and scaled bias keep, and the output
    layer's -ln 2 = 1 / -log2(e) removes.  In exact arithmetic this is the network unchanged
    (up to the float32 rounding of the products); with BF16 operands the rounded values are
    the scaled ones."""
    from types import SimpleNamespace
    last = len(weights.W) - 1
    W = [np.asarray(w, np.float32) for w in weights.W]
    b = [np.asarray(v, np.float32) for v in weights.b]
    W[0] = W[0] * NEG_LOG2E_F32
    W[last] = W[last] * NEG_LN2_F32
    b = [v * NEG_LOG2E_F32 if l < last else v for l, v in enumerate(b)]
    return SimpleNamespace(hidden=weights.hidden, W=W, b=b, act_scale=weights.act_scale,
                           w_scale=weights.w_scale, seed=weights.seed, n_in=weights.n_in,
                           flags=weights.flags, exp2_folded=True)


def silu_exp2(a):
    """-log2(e) SiLU(x) from a = -log2(e) x: a / (1 + 2^a)."""
    with np.errstate(over="ignore"):
        return a / (1.0 + np.exp2(a))


def velocity_fp8_exp2(weights, x, t, condf):
    """The velocity network evaluated as PREC_FP8_EXP2: the network of fold_exp2 (every
    pre-activation a' = -log2(e) a, scaled activation -log2(e) SiLU(a) = silu_exp2(a')) with
    PREC_FP8's operand roundings, except that an activation entering one of the e4m3 hidden
    layers is halved before that layer divides it by its activation scale and rounds it, and
    the layer's exact sum is doubled with its scales: with e4m3's limit of 448 the halved value
    keeps the headroom of the plain SiLU (|log2(e) / 2| < 1), and since the halving and the
    doubling are exact, the network is unchanged in exact arithmetic.  The last hidden layer's
    activation enters the BF16 output layer unhalved (whose -ln 2 undoes -log2(e))."""
    f = fold_exp2(weights)
    last = len(f.W) - 1
    n = x.shape[0]
    h = np.concatenate([x, np.full((n, 1), float(t)), condf], axis=1)
    for l in range(last + 1):
        W = f.W[l].astype(np.float64)
        b = f.b[l].astype(np.float64)
        if 0 < l < last:
            sa, sw = float(f.act_scale[l]), float(f.w_scale[l])
            a = (round_e4m3(h / sa) @ round_e4m3(W / sw).T) * (2.0 * sa * sw) + b
        else:
            a = round_bf16(h) @ round_bf16(W).T + b
        if l == last:
            return a
        y = silu_exp2(a)
        h = 0.5 * y if l + 1 < last else y


def velocity(weights, x, t, condf, precision=PREC_FP64):
    """v_theta(x, t | c) for a batch: x [n,5], t scalar, condf [n,4] -> [n,5].
    Layers: Linear(10,H) SiLU, 3 x (Linear(H,H) SiLU), Linear(H,5); the input of the first
    layer is [x, t, condition].  Weights of the residual network (those with an embedding
    width `emb`) go to film_velocity.  PREC_BF16_EXP2: the network of fold_exp2 with BF16
    operands; PREC_FP8_EXP2: velocity_fp8_exp2."""
    if getattr(weights, "emb", None) is not None:
        return film_velocity(weights, x, t, condf, precision)
    if precision == PREC_FP8_EXP2:
        return velocity_fp8_exp2(weights, x, t, condf)
    if precision == PREC_BF16_EXP2:
        weights, precision = fold_exp2(weights), PREC_BF16
    act = silu_exp2 if getattr(weights, "exp2_folded", False) else silu
    n = x.shape[0]
    h = np.concatenate([x, np.full((n, 1), float(t)), condf], axis=1)
    L = len(weights.W)
    for l in range(L):
        h = layer_affine(weights, l, h, precision)
        if l < L - 1:
            h = act(h)
    return h


def sample_raw(weights, cond, K: int, z: np.ndarray, precision=PREC_FP64) -> np.ndarray:
    """Integrate dx/dt = v(x, t) from x(0) = z with K explicit Euler steps, t_k = k / K.
    z: [5][n].  Returns x_K as [n, 5] FP64."""
    z = np.asarray(z, np.float64)
    if z.ndim != 2 or z.shape[0] != 5:
        raise ValueError("noise must have layout [5][n]")
    x = z.T.copy()
    condf = condition_features(cond)
    dt = 1.0 / K
    for k in range(K):
        x = x + dt * velocity(weights, x, k * dt, condf, precision)
    return x


def rk4_solve(f, x0, K: int):
    """Classic fourth-order Runge-Kutta over [0, 1] in K uniform steps of h = 1/K for
    dx/dt = f(x, t): each step takes slopes k1 = f(x, t), k2 = f(x + h k1 / 2, t + h / 2),
    k3 = f(x + h k2 / 2, t + h / 2), k4 = f(x + h k3, t + h) and sets
    x <- x + h (k1 + 2 k2 + 2 k3 + k4) / 6 (the integrator the paper times its sampler with:
    section "Convergence and Performance", 12 steps)."""
    x = np.array(x0, np.float64, copy=True)
    h = 1.0 / K
    for k in range(K):
        t = k * h
        k1 = f(x, t)
        k2 = f(x + 0.5 * h * k1, t + 0.5 * h)
        k3 = f(x + 0.5 * h * k2, t + 0.5 * h)
        k4 = f(x + h * k3, t + h)
        x = x + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return x


def sample_raw_rk4(weights, cond, K: int, z: np.ndarray, precision=PREC_FP64) -> np.ndarray:
    """The sampler ODE of eq. 8 (x(0) = z ~ N(0, I), dx/dt = v(x, t | c)) integrated with
    `rk4_solve` in K steps.  z: [5][n].  Returns x(1) as [n, 5] FP64."""
    z = np.asarray(z, np.float64)
    if z.ndim != 2 or z.shape[0] != 5:
        raise ValueError("noise must have layout [5][n]")
    condf = condition_features(cond)
    return rk4_solve(lambda x, t: velocity(weights, x, t, condf, precision), z.T, K)


OUTWARD = np.array([[0.0, -1.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])


def decode(raw, xy: bool = False) -> dict:
    """Exit record from the network output (paper eq. 11; the target layout is
    a0 = 2r - 1, (a1, a2) = exit direction, a3 = ln(path / L), a4 = face - 1.5).

    face = number of the thresholds -1, 0, 1 that a4 reaches (clamped to 0..3);
    pos = clamp((a0 + 1) / 2, 0, 1); direction = (a1, a2) normalised (outward normal of the
    face if the norm is below 1e-6), its normal component reflected if it points into the
    cell; path = exp(a3).  In XY geometry (xy=True) the direction is a projection: it is kept
    when its norm is at most 1 and scaled to norm 1 otherwise.  Also returns per-sample flags:
    bit0 pos clamped, bit1 direction reflected, bit2 zero-norm direction.

    Eq. 11 is defined on the range of the targets (|a| <= 16: a0, a1, a2 in [-1, 1], a4 in
    [-2, 2], ln path above about -16); a state with a component beyond 32 in magnitude, or not
    finite, is rejected: face -1, the other fields 0, flags = 8 (bit3)."""
    raw = np.asarray(raw, np.float64)
    with np.errstate(invalid="ignore"):
        rejected = ~(np.abs(raw).max(axis=1) <= 32.0) | ~np.isfinite(raw).all(axis=1)
    raw = np.where(rejected[:, None], 0.0, raw)
    a0, a1, a2, a3, a4 = (raw[:, i] for i in range(5))
    face = (a4 >= -1.0).astype(np.int32) + (a4 >= 0.0) + (a4 >= 1.0)
    p = (a0 + 1.0) / 2.0
    flags = np.zeros(raw.shape[0], np.int32)
    flags |= ((p < 0.0) | (p > 1.0)).astype(np.int32)
    pos = np.clip(p, 0.0, 1.0)
    nrm = np.hypot(a1, a2)
    small = nrm < 1e-6
    nout = OUTWARD[face]
    safe = np.where(small, 1.0, nrm)
    if xy:
        safe = np.where(small, 1.0, np.maximum(nrm, 1.0))
    u = np.where(small, nout[:, 0], a1 / safe)
    v = np.where(small, nout[:, 1], a2 / safe)
    dn = u * nout[:, 0] + v * nout[:, 1]
    inward = dn < 0.0
    u = np.where(inward, u - 2.0 * dn * nout[:, 0], u)
    v = np.where(inward, v - 2.0 * dn * nout[:, 1], v)
    flags |= inward.astype(np.int32) << 1
    flags |= small.astype(np.int32) << 2
    length = np.exp(a3)
    face = np.where(rejected, -1, face).astype(np.int32)
    pos, u, v, length = (np.where(rejected, 0.0, a) for a in (pos, u, v, length))
    flags = np.where(rejected, 8, flags).astype(np.int32)
    return dict(face=face, pos=pos, u=u, v=v, len=length, flags=flags)


# ----------------------------------------------------------------------------------------
# transport composition with a pluggable second stage (paper "Transport Algorithm", stages
# 1-4): the analog walk or the generative sampler (network of eq. 8 + decoding of eq. 11)
# ----------------------------------------------------------------------------------------

def _setup_composition(L):
    P = ctypes.c_void_p
    if getattr(L, "_composition_ready", False):
        return
    L.orc_noise_ids.argtypes = [ctypes.c_uint64, P, ctypes.c_int64, P]
    L.orc_walk_ids.argtypes = [P, P, P, P, P, P, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, P,
                               P, P, P, P, P]
    L.orc_split_ids.argtypes = [P, P, P, P, P, P, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, P,
                                P, P, P, P, P, P, P]
    L.orc_birth_states.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, P, P,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, P, P, P, P, P]
    L._composition_ready = True


def noise_ids(seed: int, ids) -> np.ndarray:
    """z ~ N(0, I_5) of the random streams ids (Philox + Box-Muller, as `noise`), [5][n]."""
    L = lib()
    _setup_composition(L)
    ids = np.ascontiguousarray(ids, np.uint64)
    z = np.zeros((5, ids.size))
    L.orc_noise_ids(seed, _p(ids), ids.size, _p(z))
    return z


def _canon_arrays(cond):
    f = lambda a: np.ascontiguousarray(a, np.float64)
    return [f(cond["tau"]), f(cond["c"]), f(cond["y_in"]), f(cond["u"]), f(cond["sin_th"]), f(cond["aspect"])]


def walk_ids(cond, seed: int, ids, xy: bool) -> dict:
    """Mode-C analog walks of canonical transmissions with FP64 conditions (dict with tau, c,
    y_in, u, sin_th, aspect) and random streams ids."""
    L = lib()
    _setup_composition(L)
    ids = np.ascontiguousarray(ids, np.uint64)
    n = ids.size
    arrs = _canon_arrays(cond)
    out = dict(face=np.zeros(n, np.int32), pos=np.zeros(n), u=np.zeros(n), v=np.zeros(n), len=np.zeros(n))
    L.orc_walk_ids(*(_p(a) for a in arrs), int(xy), n, seed, _p(ids), _p(out["face"]), _p(out["pos"]),
                   _p(out["u"]), _p(out["v"]), _p(out["len"]))
    return out


def split_ids(cond, seed: int, ids, xy: bool) -> dict:
    """First-flight split (uncollided_split) of canonical transmissions with FP64 conditions and
    random streams ids; also `margin` = |xi - exp(-c tau d_b)| of each decision."""
    L = lib()
    _setup_composition(L)
    ids = np.ascontiguousarray(ids, np.uint64)
    n = ids.size
    arrs = _canon_arrays(cond)
    out = dict(flag=np.zeros(n, np.int32), face=np.zeros(n, np.int32), pos=np.zeros(n), u=np.zeros(n),
               v=np.zeros(n), len=np.zeros(n), margin=np.zeros(n))
    L.orc_split_ids(*(_p(a) for a in arrs), int(xy), n, seed, _p(ids), _p(out["flag"]), _p(out["face"]),
                    _p(out["pos"]), _p(out["u"]), _p(out["v"]), _p(out["len"]), _p(out["margin"]))
    return out


def stage2_analog(cond, seed, ids, xy):
    """Stage 2 by the analog walk (orc_transport's own second stage)."""
    e = walk_ids(cond, seed, ids, xy)
    e["margin"] = np.full(len(e["face"]), np.inf)
    return e


def stage2_generative(weights, K: int, integrator: str = "euler", precision=PREC_FP64):
    """Stage 2 by the generative sampler: noise z of the transmission's random stream (Philox
    counter (id lo, id hi, j, 1)), the ODE of eq. 8 integrated over K steps (explicit Euler or
    classic RK4) through the velocity network `weights`, and the decoder of eq. 11.  A model
    fitted on collided crossings (flags bit 1) first takes the first-flight split: uncollided
    crossings exit at the end of their entry ray, only the others are sampled.  The network's
    condition is (ln tau, c, 2 y_in - 1, sin theta) in the canonical frame, plus ln A for an
    11-input model of rectangular cells or omega_x for an XY-geometry model.  Returns the exits
    and `margin`: the smallest distance of a decision from its threshold (a4 from the face
    thresholds -1, 0, 1, the largest |a| from the rejection bound 32, the split's xi from its
    probability), which bounds where a computation in another precision could decide
    differently."""
    from types import SimpleNamespace
    collided = bool(int(getattr(weights, "flags", 0)) & 2)
    xy_model = bool(int(getattr(weights, "flags", 0)) & 1)
    n_in = int(getattr(weights, "n_in", 10))

    def f(cond, seed, ids, xy):
        n = len(ids)
        out = dict(face=np.zeros(n, np.int32), pos=np.zeros(n), u=np.zeros(n), v=np.zeros(n),
                   len=np.zeros(n), margin=np.full(n, np.inf))
        todo = np.arange(n)
        if collided:
            sp = split_ids(cond, seed, ids, xy)
            unc = sp["flag"] == 1
            for k in ("face", "pos", "u", "v", "len", "margin"):
                out[k][unc] = sp[k][unc]
            out["margin"][~unc] = sp["margin"][~unc]
            todo = np.nonzero(~unc)[0]
        if todo.size == 0:
            return out
        c_ = SimpleNamespace(log_tau=np.log(cond["tau"][todo]), c=cond["c"][todo], y_in=cond["y_in"][todo],
                             sin_th=cond["sin_th"][todo], log_aspect=None, omega_x=None)
        if xy_model:
            c_.omega_x = cond["u"][todo]
        elif n_in == 11:
            c_.log_aspect = np.log(cond["aspect"][todo])
        z = noise_ids(seed, np.asarray(ids, np.uint64)[todo])
        raw = (sample_raw_rk4 if integrator == "rk4" else sample_raw)(weights, c_, K, z, precision)
        d = decode(raw, xy=xy)
        for k in ("face", "pos", "u", "v", "len"):
            out[k][todo] = d[k]
        with np.errstate(invalid="ignore"):
            m_face = np.min(np.abs(raw[:, 4:5] - np.array([[-1.0, 0.0, 1.0]])), axis=1)
            m_rej = np.abs(np.abs(raw).max(axis=1) - 32.0)
        out["margin"][todo] = np.minimum(out["margin"][todo], np.minimum(m_face, m_rej))
        return out
    return f


def _rot(k, a, b):
    """Rotation of the vector (a, b) by k quarter turns counter-clockwise (k per element)."""
    k = np.asarray(k) & 3
    ra = np.select([k == 0, k == 1, k == 2], [a, -b, -a], b)
    rb = np.select([k == 0, k == 1, k == 2], [b, a, -b], -a)
    return ra, rb


def transport_composed(problem, seed: int, hist, stage2, w_margin: float = 1e-5) -> dict:
    """Cell-to-cell transport of the histories `hist` (ids below 2^32), every cell transmission
    sampled by `stage2(cond, seed, ids, xy)`, in the order of the paper's transport algorithm,
    all particles of a step at once:
      births: source sampling and, for a volumetric source, the first leg in the birth cell by
        the analog walk (tallied; orc_birth_states);
      stage 4 after every visit: a rejected sample (face -1) or a weight below w_min ends the
        history (weight to the cutoff tally); otherwise the move to the neighbour through the
        exit face (entry height = exit position), or leakage / specular reflection at the
        domain boundary; a history reaching cell visit max_visits ends there (cutoff);
      stage 1: the entry face e turned to the canonical left face by (e + 1) mod 4 quarter turns,
        the entry face taken as the unit of length (tau * h_e / L, aspect w_e / h_e);
      stage 2: stage2 with random stream id h + 2^32 * (cell visit);
      stage 3: FP64 attenuation w_out = w e^{-sigma_a l} (eq. 5), deposit (eq. 6), track-length
        flux (eq. 7; w l / V when sigma_a = 0) and the path tallies, l = the physical length.
    Returns per-cell sums over the histories (flux, absorbed, leak, cutoff, wpath, path, visits,
    rejected_w, rejected_n), the number of transmissions (`events`, birth legs included) and
    `at_risk`: the histories with a decision within its margin (stage 2's margin below 1e-4, or
    a weight within w_margin relative of w_min)."""
    L_ = lib()
    _setup_composition(L_)
    P = problem
    nc = P.n_cells
    Lx = P.L
    Ly = P.Ly if getattr(P, "Ly", 0.0) > 0 else P.L
    xy = bool(getattr(P, "xy", False))
    max_visits = int(getattr(P, "max_visits", 0)) or (1 << 24)
    tau = np.ascontiguousarray(P.tau, np.float64)
    cc = np.ascontiguousarray(P.c, np.float64)
    T = {k: np.zeros(nc) for k in ("flux", "absorbed", "leak", "cutoff", "wpath", "path", "visits",
                                   "rejected_w", "rejected_n")}
    hist = np.unique(np.asarray(hist, np.int64))
    # births, per contiguous run of history ids
    runs = np.split(hist, np.nonzero(np.diff(hist) != 1)[0] + 1) if hist.size else []
    states, sc = [], np.zeros(3)
    for r in runs:
        st = np.zeros((9, r.size))
        pt = np.zeros((3, nc))
        L_.orc_birth_states(P.nx, P.ny, Lx, float(getattr(P, "Ly", 0.0)), _p(tau), _p(cc), P.src_x0, P.src_y0,
                            P.src_nx, P.src_ny, int(P.reflect), int(getattr(P, "src_face", -1)), int(xy),
                            P.w_min, seed, int(r[0]), int(r[-1]) + 1, _p(st), _p(T["flux"]), _p(T["absorbed"]),
                            _p(pt), _p(sc))
        T["wpath"] += pt[0]
        T["path"] += pt[1]
        T["visits"] += pt[2]
        states.append(st)
    st = np.concatenate(states, axis=1) if states else np.zeros((9, 0))
    events = sc[2]
    at_entry = st[0] == 1.0
    cell = st[1].astype(np.int64)
    face = st[2].astype(np.int64)          # exit face after a visit / entry face at an entry
    pos = st[3].copy()                      # exit position / canonical entry height
    gx, gy, w = st[4].copy(), st[5].copy(), st[6].copy()
    ev = st[7].astype(np.int64)
    h = hist.copy()
    at_risk = set()
    V = Lx * Ly
    while h.size:
        # ---- stage 4 for the particles that have just finished a visit
        done = ~at_entry
        entry = face.copy()
        y_in = pos.copy()
        alive = np.ones(h.size, bool)
        if done.any():
            i = np.nonzero(done)[0]
            near = np.abs(w[i] - P.w_min) <= w_margin * P.w_min
            at_risk.update(h[i[near]].tolist())
            rej = face[i] < 0
            low = (~rej) & (w[i] < P.w_min)
            np.add.at(T["cutoff"], cell[i[rej | low]], w[i[rej | low]])
            np.add.at(T["rejected_w"], cell[i[rej]], w[i[rej]])
            np.add.at(T["rejected_n"], cell[i[rej]], 1.0)
            alive[i[rej | low]] = False
            mv = i[~(rej | low)]
            f = face[mv]
            ci, cj = cell[mv] % P.nx, cell[mv] // P.nx
            ni = ci + np.where(f == 1, 1, np.where(f == 3, -1, 0))
            nj = cj + np.where(f == 2, 1, np.where(f == 0, -1, 0))
            out = (ni < 0) | (nj < 0) | (ni >= P.nx) | (nj >= P.ny)
            if not P.reflect:
                np.add.at(T["leak"], cell[mv[out]], w[mv[out]])
                alive[mv[out]] = False
            else:
                r_ = mv[out]
                entry[r_] = face[r_]
                y_in[r_] = 1.0 - pos[r_]
                horiz = (face[r_] == 0) | (face[r_] == 2)
                gy[r_] = np.where(horiz, -gy[r_], gy[r_])
                gx[r_] = np.where(horiz, gx[r_], -gx[r_])
            inn = mv[~out]
            cell[inn] = nj[~out] * P.nx + ni[~out]
            entry[inn] = (face[inn] + 2) & 3
            y_in[inn] = pos[inn]
            moved = mv[alive[mv]]
            ev[moved] += 1
            cap = moved[ev[moved] >= max_visits]
            np.add.at(T["cutoff"], cell[cap], w[cap])
            alive[cap] = False
        keep = np.nonzero(alive)[0]
        h, cell, entry, y_in, gx, gy, w, ev = (a[keep] for a in (h, cell, entry, y_in, gx, gy, w, ev))
        if not h.size:
            break
        # ---- stage 1: canonical frame of the entry face
        k = (entry + 1) & 3
        U, Vc = _rot((4 - k) & 3, gx, gy)
        odd = (entry & 1) == 1
        h_e = np.where(odd, Ly, Lx)
        w_e = np.where(odd, Lx, Ly)
        s = Vc if xy else np.clip(Vc, -1.0, 1.0)
        u0 = U if xy else np.sqrt(1.0 - s * s)
        cond = dict(tau=tau[cell] * h_e / Lx, c=cc[cell], y_in=y_in, u=u0, sin_th=s, aspect=w_e / h_e)
        ids = h.astype(np.uint64) | (ev.astype(np.uint64) << np.uint64(32))
        # ---- stage 2
        e = stage2(cond, seed, ids, xy)
        events += h.size
        at_risk.update(h[e["margin"] < 1e-4].tolist())
        # ---- stage 3 (FP64)
        sig_a = (1.0 - cc[cell]) * tau[cell] / Lx
        ls = e["len"] * h_e
        dw = w * (-np.expm1(-sig_a * ls))
        with np.errstate(divide="ignore", invalid="ignore"):
            phi = np.where(sig_a > 0.0, dw / (V * sig_a), w * ls / V)
        np.add.at(T["flux"], cell, phi)
        np.add.at(T["absorbed"], cell, dw)
        np.add.at(T["wpath"], cell, w * ls)
        np.add.at(T["path"], cell, ls)
        np.add.at(T["visits"], cell, 1.0)
        w = w - dw
        # back to the global frame
        face = np.where(e["face"] >= 0, (e["face"] + k) & 3, e["face"])
        pos = e["pos"]
        gx, gy = _rot(k, e["u"], e["v"])
        at_entry = np.zeros(h.size, bool)
    T["events"] = events
    T["at_risk"] = sorted(at_risk)
    return T
