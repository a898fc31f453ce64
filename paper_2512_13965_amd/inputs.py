"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the CPU oracle.

This module holds no arithmetic of the method itself: it only draws the inputs a
caller would hand to a cell-transmission sampler (entry conditions, network
weights, Gaussian noise, transport problem descriptions) and packs the weights
into the on-disk blob that the C library parses.  Every generator takes an
explicit integer seed and uses numpy's PCG64, so any input can be re-created
from its seed alone.

Workload recipes (sizes and laws follow the paper's workloads):

* entry conditions of a cell transmission in the canonical left-entry frame
  (paper, "Network Architecture and Inputs", eq. 10, and "Transport
  Algorithm", first stage): optical side tau = sigma_t * L with
  ln tau ~ U[ln 0.1, ln 100], scattering ratio c ~ U[0, 1], entry height
  y_in ~ U(0, 1) on the left face, and a cosine-law entry direction.  For a
  flatland cosine law the pdf of theta is cos(theta)/2 on (-pi/2, pi/2), which
  makes sin(theta_in) uniform on (-1, 1); we draw sin(theta_in) directly.
* conditions of the internal (volumetric-source) model: the same ln tau and c
  laws, a birth point (x, y) uniform in the unit cell and an isotropic birth
  direction phi ~ U[0, 2 pi) given as (cos phi, sin phi) (paper, "Network
  Architecture and Inputs": the internal model is conditioned on the birth
  position and direction instead of the entry height and angle).
* velocity-network weights: fully connected n_in -> H -> H -> H -> H -> 5
  (n_in = 10 for the boundary model, 12 for the internal model),
  every weight and bias U(-1/sqrt(fan_in), +1/sqrt(fan_in)) (the usual
  default initialisation of a linear layer), float32.
* weights of the residual network with adaptive modulation (blob flag bit 2): the same
  initialisation law for every layer (input layer, embedding, the three blocks' main,
  scale and shift maps, output layer).
* noise z ~ N(0, I_5) when a caller wants to hand the sampler its noise
  explicitly (paper, "Conditional Flow Matching", eq. 8).
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass, field

import numpy as np

N_IN = 10            # boundary model: x (5), t (1), condition (4)
N_IN_RECT = 11       # boundary model of rectangular cells: x (5), t (1), condition (5)
N_IN_INTERNAL = 12   # internal (volumetric-source) model: x (5), t (1), condition (6)
N_OUT = 5   # exit state: position, cos, sin, log path, face
N_LAYERS = 5

# Residual network with adaptive modulation (blob flag bit 2): embedding width, residual
# blocks and number of time features of its input.
FILM_FLAG = 4
FILM_EMB = 32
FILM_BLOCKS = 3
N_TIME_FEATURES = 8

BLOB_MAGIC = b"GMCW0001"
BLOB_VERSION = 1
# header: magic[8], version, n_in, hidden, n_out, n_layers, flags, seed, reserved (8 x u32),
# act_scale[5] f32, w_scale[5] f32
_HDR = struct.Struct("<8s8I5f5f")

LOG_TAU_MIN = math.log(0.1)
LOG_TAU_MAX = math.log(100.0)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _open01(g: np.random.Generator, n: int) -> np.ndarray:
    """Uniform on the open interval (0, 1) in float32."""
    u = g.random(n, dtype=np.float64)
    u = np.clip(u, 2.0 ** -25, 1.0 - 2.0 ** -24)
    return u.astype(np.float32)


@dataclass
class Conditions:
    """Structure-of-arrays batch of canonical entry conditions (all float32, length n).
    log_aspect (optional): ln A of rectangular cells, A = width along the flight direction
    over the entry face's length (None: square cells).  omega_x (optional): XY geometry, the
    in-plane x component of the entry direction, sin_th then being its y component (None:
    flatland, unit in-plane direction)."""
    log_tau: np.ndarray
    c: np.ndarray
    y_in: np.ndarray
    sin_th: np.ndarray
    log_aspect: np.ndarray | None = None
    omega_x: np.ndarray | None = None

    def __len__(self) -> int:
        return int(self.log_tau.shape[0])

    def subset(self, idx) -> "Conditions":
        return Conditions(self.log_tau[idx].copy(), self.c[idx].copy(),
                          self.y_in[idx].copy(), self.sin_th[idx].copy(),
                          None if self.log_aspect is None else self.log_aspect[idx].copy(),
                          None if self.omega_x is None else self.omega_x[idx].copy())


def transmission_conditions(n: int, seed: int, log_tau_range=(LOG_TAU_MIN, LOG_TAU_MAX),
                            c_range=(0.0, 1.0), log_aspect_range=None) -> Conditions:
    """Mixed-cell batch: ln tau ~ U[range], c ~ U[range], y_in ~ U(0,1), cosine-law entry;
    with log_aspect_range, rectangular cells with ln A ~ U[range] (drawn after the rest, so the
    square-cell fields are those of the same seed without it)."""
    g = rng(seed)
    lo, hi = log_tau_range
    log_tau = (lo + (hi - lo) * g.random(n)).astype(np.float32)
    c = (c_range[0] + (c_range[1] - c_range[0]) * g.random(n)).astype(np.float32)
    y_in = _open01(g, n)
    sin_th = (2.0 * _open01(g, n).astype(np.float64) - 1.0).astype(np.float32)
    la = None
    if log_aspect_range is not None:
        a0, a1 = log_aspect_range
        la = (a0 + (a1 - a0) * g.random(n)).astype(np.float32)
    return Conditions(log_tau, c, y_in, sin_th, la)


def _xy_entry(g, n):
    """Entry directions of isotropic incident flux in three dimensions, projected on the plane:
    cosine to the inward normal sqrt(xi), azimuth psi about it; (omega_x, omega_y) =
    (sqrt(xi), sqrt(1 - xi) cos psi)."""
    xi = _open01(g, n).astype(np.float64)
    psi = 2.0 * math.pi * _open01(g, n).astype(np.float64)
    return np.sqrt(xi).astype(np.float32), (np.sqrt(1.0 - xi) * np.cos(psi)).astype(np.float32)


def xy_conditions(n: int, seed: int, log_tau_range=(LOG_TAU_MIN, LOG_TAU_MAX),
                  c_range=(0.0, 1.0)) -> Conditions:
    """Mixed-cell batch in XY geometry: ln tau, c and y_in as transmission_conditions, entry
    directions of isotropic incident flux on the sphere (projected)."""
    g = rng(seed)
    lo, hi = log_tau_range
    log_tau = (lo + (hi - lo) * g.random(n)).astype(np.float32)
    c = (c_range[0] + (c_range[1] - c_range[0]) * g.random(n)).astype(np.float32)
    y_in = _open01(g, n)
    ox, oy = _xy_entry(g, n)
    return Conditions(log_tau, c, y_in, oy, None, ox)


def fixed_xy_conditions(n: int, tau: float, c: float, seed: int) -> Conditions:
    """One material for every particle, XY geometry; y_in ~ U(0,1), isotropic incident flux."""
    g = rng(seed)
    y_in = _open01(g, n)
    ox, oy = _xy_entry(g, n)
    return Conditions(np.full(n, np.float32(math.log(tau)), np.float32),
                      np.full(n, np.float32(c), np.float32), y_in, oy, None, ox)


def fixed_cell_conditions(n: int, tau: float, c: float, seed: int) -> Conditions:
    """One material (tau, c) for every particle; y_in ~ U(0,1), cosine-law entry."""
    g = rng(seed)
    y_in = _open01(g, n)
    sin_th = (2.0 * _open01(g, n).astype(np.float64) - 1.0).astype(np.float32)
    return Conditions(np.full(n, np.float32(math.log(tau)), np.float32),
                      np.full(n, np.float32(c), np.float32), y_in, sin_th)


@dataclass
class InternalConditions:
    """Structure-of-arrays batch of birth conditions for the internal (volumetric-source) model:
    optical side ln tau, scattering ratio c, birth position (x, y) in the unit cell and birth
    direction (cos phi, sin phi) in the cell's own frame (all float32, length n)."""
    log_tau: np.ndarray
    c: np.ndarray
    x: np.ndarray
    y: np.ndarray
    cos_phi: np.ndarray
    sin_phi: np.ndarray

    def __len__(self) -> int:
        return int(self.log_tau.shape[0])

    def subset(self, idx) -> "InternalConditions":
        return InternalConditions(*(a[idx].copy() for a in (self.log_tau, self.c, self.x, self.y,
                                                             self.cos_phi, self.sin_phi)))


def internal_conditions(n: int, seed: int, log_tau_range=(LOG_TAU_MIN, LOG_TAU_MAX),
                        c_range=(0.0, 1.0)) -> InternalConditions:
    """Mixed-cell births: ln tau, c uniform on their ranges, position uniform in the cell,
    isotropic direction (phi uniform on [0, 2 pi))."""
    g = rng(seed)
    lo, hi = log_tau_range
    log_tau = (lo + (hi - lo) * g.random(n)).astype(np.float32)
    c = (c_range[0] + (c_range[1] - c_range[0]) * g.random(n)).astype(np.float32)
    x = _open01(g, n)
    y = _open01(g, n)
    phi = 2.0 * math.pi * g.random(n)
    return InternalConditions(log_tau, c, x, y, np.cos(phi).astype(np.float32),
                              np.sin(phi).astype(np.float32))


def fixed_internal_conditions(n: int, tau: float, c: float, seed: int) -> InternalConditions:
    """One material for every birth; uniform position, isotropic direction."""
    b = internal_conditions(n, seed)
    b.log_tau[:] = np.float32(math.log(tau))
    b.c[:] = np.float32(c)
    return b


def normal_incidence_conditions(n: int, tau: float, c: float, seed: int) -> Conditions:
    """A beam along +x (sin theta = 0) at uniform entry height."""
    g = rng(seed)
    return Conditions(np.full(n, np.float32(math.log(tau)), np.float32),
                      np.full(n, np.float32(c), np.float32), _open01(g, n),
                      np.zeros(n, np.float32))


def noise(n: int, seed: int) -> np.ndarray:
    """Explicit N(0, I_5) noise, float32, layout [5][n]."""
    return rng(seed).standard_normal((N_OUT, n)).astype(np.float32)


# --------------------------------------------------------------------------------------
# velocity-network weights
# --------------------------------------------------------------------------------------

def layer_dims(hidden: int, n_in: int = N_IN):
    return [(hidden, n_in), (hidden, hidden), (hidden, hidden), (hidden, hidden), (N_OUT, hidden)]


@dataclass
class Weights:
    """Float32 weights W[l] of shape [out, in] (row-major) and biases b[l] of shape [out]."""
    hidden: int
    W: list
    b: list
    act_scale: np.ndarray = field(default_factory=lambda: np.ones(N_LAYERS, np.float32))
    w_scale: np.ndarray = field(default_factory=lambda: np.ones(N_LAYERS, np.float32))
    seed: int = 0
    n_in: int = N_IN          # 10: boundary model, 11: rectangular / XY boundary model, 12: internal
    flags: int = 0            # bit 0: XY geometry (11 inputs, fifth condition feature omega_x)

    def n_params(self) -> int:
        return int(sum(w.size + bb.size for w, bb in zip(self.W, self.b)))


def film_layer_dims(hidden: int, emb: int = FILM_EMB, n_in: int = N_IN, blocks: int = FILM_BLOCKS):
    """[out, in] of every layer of the residual network in blob order: the input layer over
    [x (5), time features (8), condition (n_in - 6)], the embedding over [time features,
    condition], then per block the main H x H map and the E -> H scale and shift maps, and the
    output layer."""
    n_c = n_in - 6
    dims = [(hidden, 5 + N_TIME_FEATURES + n_c), (emb, N_TIME_FEATURES + n_c)]
    for _ in range(blocks):
        dims += [(hidden, hidden), (hidden, emb), (hidden, emb)]
    return dims + [(N_OUT, hidden)]


@dataclass
class FilmWeights:
    """Float32 layers W[l] [out, in] and biases b[l] [out] of the residual network with
    adaptive modulation, in the order of film_layer_dims."""
    hidden: int
    emb: int
    W: list
    b: list
    seed: int = 0
    n_in: int = N_IN
    flags: int = FILM_FLAG    # bit 2 set; bits 0 and 1 as for Weights

    @property
    def blocks(self) -> int:
        return (len(self.W) - 3) // 3

    def n_params(self) -> int:
        return int(sum(w.size + bb.size for w, bb in zip(self.W, self.b)))


def random_film_weights(hidden: int, seed: int, emb: int = FILM_EMB, blocks: int = FILM_BLOCKS,
                        n_in: int = N_IN, flags: int = 0) -> FilmWeights:
    """Seeded random-init residual network, U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every
    weight and bias."""
    g = rng(seed)
    W, b = [], []
    for (o, i) in film_layer_dims(hidden, emb, n_in, blocks):
        bound = 1.0 / math.sqrt(i)
        W.append(g.uniform(-bound, bound, size=(o, i)).astype(np.float32))
        b.append(g.uniform(-bound, bound, size=(o,)).astype(np.float32))
    return FilmWeights(hidden, emb, W, b, seed, n_in, int(flags) | FILM_FLAG)


def pow2_ceil_scale(amax: float, fmax: float = 448.0) -> float:
    """Smallest power of two s with amax / s <= fmax (1.0 for amax == 0)."""
    if amax <= 0.0:
        return 1.0
    return float(2.0 ** math.ceil(math.log2(amax / fmax)))


def random_weights(hidden: int, seed: int, act_scale: float = 2.0 ** -5, n_in: int = N_IN,
                   flags: int = 0) -> Weights:
    """Seeded random-init network, U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for W and b.

    The per-layer FP8 scales are stored with the weights: the weight scale is the
    power of two that brings max|W_l| under the e4m3 maximum 448, and the
    activation scale of every layer is the constant `act_scale` (a power of two
    chosen by the model's author; the hidden activations of such a network stay
    well inside 448 * act_scale).
    """
    g = rng(seed)
    W, b = [], []
    for (o, i) in layer_dims(hidden, n_in):
        bound = 1.0 / math.sqrt(i)
        W.append(g.uniform(-bound, bound, size=(o, i)).astype(np.float32))
        b.append(g.uniform(-bound, bound, size=(o,)).astype(np.float32))
    w_scale = np.array([pow2_ceil_scale(float(np.abs(w).max())) for w in W], np.float32)
    a_scale = np.full(N_LAYERS, np.float32(act_scale), np.float32)
    return Weights(hidden, W, b, a_scale, w_scale, seed, n_in, flags)


def pack_blob(w) -> bytes:
    """Serialise to the versioned little-endian blob read by gmc_model_create().  A residual
    network (FilmWeights) sets flag bit 2 and stores its block count in the n_layers field and
    its embedding width in the reserved field; its scale fields are 1."""
    if isinstance(w, FilmWeights):
        hdr = _HDR.pack(BLOB_MAGIC, BLOB_VERSION, w.n_in, w.hidden, N_OUT, w.blocks,
                        int(w.flags) | FILM_FLAG, int(w.seed) & 0xFFFFFFFF, w.emb,
                        *([1.0] * 5), *([1.0] * 5))
    else:
        hdr = _HDR.pack(BLOB_MAGIC, BLOB_VERSION, w.n_in, w.hidden, N_OUT, N_LAYERS, int(w.flags),
                        int(w.seed) & 0xFFFFFFFF, 0,
                        *[float(x) for x in w.act_scale], *[float(x) for x in w.w_scale])
    parts = [hdr]
    for W, b in zip(w.W, w.b):
        parts.append(np.ascontiguousarray(W, np.float32).tobytes())
        parts.append(np.ascontiguousarray(b, np.float32).tobytes())
    return b"".join(parts)


def unpack_blob(blob: bytes):
    fields = _HDR.unpack_from(blob, 0)
    magic, version, n_in, hidden, n_out, n_layers, flags, seed, res = fields[:9]
    film = bool(flags & FILM_FLAG)
    if magic != BLOB_MAGIC or version != BLOB_VERSION or n_in not in (N_IN, N_IN_RECT, N_IN_INTERNAL) \
            or n_out != N_OUT or (n_layers != N_LAYERS and not film):
        raise ValueError("not a GMC weights blob of a supported version")
    act = np.array(fields[9:14], np.float32)
    wsc = np.array(fields[14:19], np.float32)
    off = _HDR.size
    W, b = [], []
    dims = film_layer_dims(hidden, res, n_in, n_layers) if film else layer_dims(hidden, n_in)
    for (o, i) in dims:
        W.append(np.frombuffer(blob, np.float32, o * i, off).reshape(o, i).copy())
        off += 4 * o * i
        b.append(np.frombuffer(blob, np.float32, o, off).copy())
        off += 4 * o
    if off != len(blob):
        raise ValueError("weights blob has trailing or missing bytes")
    if film:
        return FilmWeights(hidden, res, W, b, seed, n_in, flags)
    return Weights(hidden, W, b, act, wsc, seed, n_in, flags)


def save_blob(w: Weights, path: str) -> None:
    with open(path, "wb") as f:
        f.write(pack_blob(w))


def load_blob(path: str) -> Weights:
    with open(path, "rb") as f:
        return unpack_blob(f.read())


# --------------------------------------------------------------------------------------
# transport problems (2-D grids of square cells)
# --------------------------------------------------------------------------------------

@dataclass
class Problem:
    """A 2-D grid of nx * ny cells of width L (along x) and height Ly (0: square, Ly = L),
    per-cell (tau, c), a source.

    Cell (i, j) has linear index j * nx + i (i along x).  tau = sigma_t * L.
    src_face = -1: isotropic unit source uniform over the source block's cells; src_face = f in
    0..3 (bottom, right, top, left): isotropic incident flux on that side of the domain over the
    source strip's cells (the block must be one cell thick along that side).
    """
    nx: int
    ny: int
    L: float
    tau: np.ndarray       # float64 [ny * nx]
    c: np.ndarray         # float64 [ny * nx]
    src_x0: int
    src_y0: int
    src_nx: int
    src_ny: int
    reflect: bool = False
    w_min: float = 1e-6
    src_face: int = -1
    Ly: float = 0.0
    xy: bool = False          # XY geometry: directions on the sphere (eq. 1), invariant along z
    max_visits: int = 0       # a history is cut off before this cell visit number (0: 2^24)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny


def checkerboard_problem(n: int = 32, tau=(0.5, 50.0), c=(0.5, 0.99), src: int = 4,
                         L: float = 1.0, reflect: bool = False) -> Problem:
    """n x n unit cells; (tau[0], c[0]) where i + j is even, (tau[1], c[1]) where odd;
    isotropic source in the central src x src cells; vacuum boundaries."""
    i = np.arange(n)[None, :]
    j = np.arange(n)[:, None]
    odd = ((i + j) % 2).astype(bool).reshape(-1)
    t = np.where(odd, tau[1], tau[0]).astype(np.float64)
    cc = np.where(odd, c[1], c[0]).astype(np.float64)
    s0 = (n - src) // 2
    return Problem(n, n, L, t, cc, s0, s0, src, src, reflect)


def homogeneous_problem(n: int, tau: float, c: float, reflect: bool, src_all: bool = True,
                        L: float = 1.0) -> Problem:
    t = np.full(n * n, tau, np.float64)
    cc = np.full(n * n, c, np.float64)
    if src_all:
        return Problem(n, n, L, t, cc, 0, 0, n, n, reflect)
    s0 = (n - max(1, n // 8)) // 2
    return Problem(n, n, L, t, cc, s0, s0, max(1, n // 8), max(1, n // 8), reflect)


def random_problem(seed: int, side_range=(16, 128), log_tau_range=(math.log(0.1), math.log(200.0)),
                   hist_log10_range=(4.0, 7.0)):
    """A serving request: grid side ~ U{16..128}, per-cell ln tau ~ U[range], c ~ U[0,1],
    central (side/8)^2 source block, histories log-uniform in [1e4, 1e7].
    Returns (problem, n_histories)."""
    g = rng(seed)
    n = int(g.integers(side_range[0], side_range[1] + 1))
    lo, hi = log_tau_range
    tau = np.exp(lo + (hi - lo) * g.random(n * n))
    c = g.random(n * n)
    s = max(1, n // 8)
    s0 = (n - s) // 2
    nh = int(round(10.0 ** (hist_log10_range[0] + (hist_log10_range[1] - hist_log10_range[0])
                            * g.random())))
    return Problem(n, n, 1.0, tau, c, s0, s0, s, s), nh


def _from_sigmas(sig_a: np.ndarray, sig_s: np.ndarray, L: float):
    """Per-cell (tau = sigma_t L, c = sigma_s / sigma_t) from cross sections in 1/cm."""
    sig_t = sig_a + sig_s
    return sig_t * L, np.where(sig_t > 0, sig_s / np.where(sig_t > 0, sig_t, 1.0), 1.0)


def lattice_problem(cells_per_cm: int = 16, cells_per_cm_y: int | None = None) -> Problem:
    """Heterogeneous lattice with the cross sections of the paper's first benchmark ("Benchmark
    Performance"): a 7 x 7 cm square, 112 x 112 cells at 16 cells per cm; scattering background
    sigma_a = 0, sigma_s = 1 /cm; absorbing blocks sigma_a = 9.5, sigma_s = 0.5 /cm; an
    isotropic volumetric source in the central 1 x 1 cm block; vacuum boundaries.

    The paper's figure with the layout is not part of its text; the layout here is defined by
    this library: the 1 x 1 cm blocks (I, J), I, J in 1..5 with I + J even, other than the
    central source block (3, 3), are absorbers (a periodic array, twelve blocks).
    cells_per_cm_y (default: cells_per_cm) gives rectangular cells of 1 / cells_per_cm by
    1 / cells_per_cm_y cm."""
    m = cells_per_cm
    my = m if cells_per_cm_y is None else cells_per_cm_y
    n, ny = 7 * m, 7 * my
    L, Ly = 1.0 / m, 1.0 / my
    I = np.arange(n)[None, :] // m
    J = np.arange(ny)[:, None] // my
    absorber = (I >= 1) & (I <= 5) & (J >= 1) & (J <= 5) & ((I + J) % 2 == 0) & ~((I == 3) & (J == 3))
    sig_a = np.where(absorber, 9.5, 0.0).reshape(-1)
    sig_s = np.where(absorber, 0.5, 1.0).reshape(-1)
    tau, c = _from_sigmas(sig_a, sig_s, L)
    return Problem(n, ny, L, tau, c, 3 * m, 3 * my, m, my, Ly=0.0 if my == m else Ly)


HOHLRAUM_MATERIALS = {          # (sigma_a, sigma_s) in 1/cm, from the paper's second benchmark
    "black": (50.0, 50.0),      # absorbing walls
    "red": (5.0, 95.0),         # stripes
    "green": (10.0, 90.0),      # framing regions
    "blue": (95.0, 5.0),        # central absorber
    "white": (0.0, 5.0),        # near vacuum
}


def hohlraum_problem(n: int = 112) -> Problem:
    """Linearized hohlraum with the cross sections of the paper's second benchmark: a 1.3 x 1.3
    cm square on an n x n mesh (112 in the paper), driven by isotropic incident flux on the
    left side (x = 0), vacuum elsewhere.

    The layout (the paper's figure is not part of its text) is defined by this library, in cm:
    black walls along the right side (x > 1.25), the top (y > 1.25) and the bottom (y < 0.05);
    red stripes y in [0.25, 0.30] and [1.00, 1.05] for x in [0.45, 1.25]; a central blue
    absorber [0.45, 0.85]^2 inside a green frame [0.40, 0.90]^2; white elsewhere.  A cell takes
    the material at its centre."""
    L = 1.3 / n
    xc = (np.arange(n)[None, :] + 0.5) * L + np.zeros((n, 1))
    yc = (np.arange(n)[:, None] + 0.5) * L + np.zeros((1, n))
    mat = np.full((n, n), "white", dtype=object)
    inside = lambda x0, x1, y0, y1: (xc >= x0) & (xc < x1) & (yc >= y0) & (yc < y1)
    mat[inside(0.40, 0.90, 0.40, 0.90)] = "green"
    mat[inside(0.45, 0.85, 0.45, 0.85)] = "blue"
    mat[inside(0.45, 1.25, 0.25, 0.30) | inside(0.45, 1.25, 1.00, 1.05)] = "red"
    mat[(xc > 1.25) | (yc > 1.25) | (yc < 0.05)] = "black"
    sig_a = np.array([HOHLRAUM_MATERIALS[k][0] for k in mat.reshape(-1)])
    sig_s = np.array([HOHLRAUM_MATERIALS[k][1] for k in mat.reshape(-1)])
    tau, c = _from_sigmas(sig_a, sig_s, L)
    return Problem(n, n, L, tau, c, 0, 0, 1, n, False, 1e-6, 3)
