"""Pins of the oracle's transport composition (paper "Transport Algorithm", stages 1-4, with a
pluggable second stage): with the analog walk as stage 2 it must be the oracle's per-history
transport, and with a hand-built network that sends every particle straight across its cell it
must give the straight-line tallies worked out history by history."""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs

NT = 4
_T = np.array([0.3, 2.0, 0.7, 1.5, 0.5, 3.0, 0.9, 0.2, 1.1])
_C = np.array([0.9, 0.5, 0.99, 0.7, 0.8, 0.95, 0.3, 1.0, 0.6])


def _problems():
    out = [("checker8", inputs.checkerboard_problem(8, src=2)),
           ("hetero3", inputs.Problem(3, 3, 0.7, _T, _C, 1, 1, 1, 1)),
           ("rect_flat", inputs.Problem(3, 3, 0.7, _T, _C, 1, 1, 1, 1, Ly=0.35)),
           ("rect_tall", inputs.Problem(3, 3, 0.7, _T, _C, 1, 1, 1, 1, Ly=1.6)),
           ("xy", inputs.Problem(3, 3, 0.7, _T, _C, 1, 1, 1, 1, xy=True)),
           ("xy_rect", inputs.Problem(3, 3, 0.7, _T, _C, 1, 1, 1, 1, Ly=0.5, xy=True))]
    for f in range(4):
        x0, y0, nx_, ny_ = {3: (0, 0, 1, 3), 1: (2, 0, 1, 3), 0: (0, 0, 3, 1), 2: (0, 2, 3, 1)}[f]
        out.append((f"surface{f}", inputs.Problem(3, 3, 0.7, _T, _C, x0, y0, nx_, ny_, src_face=f)))
    refl = inputs.Problem(3, 3, 0.7, _T, _C, 0, 0, 3, 3, reflect=True)
    refl.max_visits = 40
    out.append(("reflect_cap", refl))
    return out


@pytest.mark.parametrize("name,prob", _problems(), ids=[p[0] for p in _problems()])
def test_analog_stage2_reproduces_history_transport(orc, name, prob):
    n = 1500
    a = orc.transport(prob, seed=5, h_begin=0, h_end=n, nthreads=NT)
    b = orc.transport_composed(prob, 5, np.arange(n), orc.stage2_analog)
    for k in ("flux", "absorbed", "wpath", "path"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-11, atol=1e-13 * n, err_msg=k)
    np.testing.assert_array_equal(b["visits"], a["visits"])
    assert b["events"] == a["events"]
    assert b["leak"].sum() == pytest.approx(a["leak"], rel=1e-12, abs=1e-12)
    assert b["cutoff"].sum() == pytest.approx(a["cutoff"], rel=1e-12, abs=1e-12)
    # a subset of the histories is the corresponding part of the sums
    c1 = orc.transport_composed(prob, 5, np.arange(0, n, 2), orc.stage2_analog)
    c2 = orc.transport_composed(prob, 5, np.arange(1, n, 2), orc.stage2_analog)
    np.testing.assert_allclose(c1["flux"] + c2["flux"], b["flux"], rtol=1e-11, atol=1e-13 * n)


def straight_network(n_in: int = 10) -> inputs.Weights:
    """K = 1 Euler from z: v = target - z, so x_1 = (2 y_in - 1, 1, 0, 0, -0.5) whatever the
    noise: the right face (a4 = -0.5), at the entry height, along +x, path 1.  Pre-activations
    are z + 100 or (2 y_in - 1) + 100, where SiLU is the identity in FP64."""
    H = 16
    W = [np.zeros((H, n_in), np.float32), np.eye(H, dtype=np.float32), np.eye(H, dtype=np.float32),
         np.eye(H, dtype=np.float32), np.zeros((5, H), np.float32)]
    b = [np.zeros(H, np.float32) for _ in range(4)] + [np.zeros(5, np.float32)]
    for d in range(5):
        W[0][d, d] = 1.0          # z_d + 100
    W[0][5, 8] = 1.0              # (2 y_in - 1) + 100
    b[0][:6] = 100.0
    W[4][0, 0], W[4][0, 5] = -1.0, 1.0              # v0 = (2y - 1) - z0
    for d, target in ((1, 1.0), (2, 0.0), (3, 0.0), (4, -0.5)):
        W[4][d, d] = -1.0
        b[4][d] = 100.0 + target                    # v_d = target - z_d
    return inputs.Weights(H, W, b, np.ones(5, np.float32), np.ones(5, np.float32), n_in=n_in)


def _straight_lines(orc, prob, seed, n):
    """Per-history reference for the straight network: after its birth a particle keeps
    crossing cells along the same direction, entering each through the face opposite its exit,
    at the same height, each visit's track one entry-face length h_e; attenuation e^{-sigma_a l},
    leakage at the domain boundary, the cutoff below w_min.  Plain per-history Python."""
    st = np.zeros((9, n))
    nc = prob.n_cells
    flux, absorbed, pt, sc = np.zeros(nc), np.zeros(nc), np.zeros((3, nc)), np.zeros(3)
    L = orc.lib()
    orc._setup_composition(L)
    L.orc_birth_states(prob.nx, prob.ny, prob.L, float(prob.Ly), orc._p(np.ascontiguousarray(prob.tau)),
                       orc._p(np.ascontiguousarray(prob.c)), prob.src_x0, prob.src_y0, prob.src_nx, prob.src_ny,
                       int(prob.reflect), int(prob.src_face), 0, prob.w_min, seed, 0, n, orc._p(st),
                       orc._p(flux), orc._p(absorbed), orc._p(pt), orc._p(sc))
    Ly = prob.Ly if prob.Ly > 0 else prob.L
    leak = 0.0
    path = pt[1].copy()
    for i in range(n):
        cell, f, w = int(st[1, i]), int(st[2, i]), st[6, i]
        ci, cj = cell % prob.nx, cell // prob.nx
        while w >= prob.w_min:
            ci += {1: 1, 3: -1}.get(f, 0)
            cj += {2: 1, 0: -1}.get(f, 0)
            if not (0 <= ci < prob.nx and 0 <= cj < prob.ny):
                leak += w
                break
            cell = cj * prob.nx + ci
            h_e = Ly if f in (1, 3) else prob.L          # entered through the face opposite f
            sig_a = (1.0 - prob.c[cell]) * prob.tau[cell] / prob.L
            dw = w * -math.expm1(-sig_a * h_e)
            flux[cell] += (dw / sig_a if sig_a > 0 else w * h_e) / (prob.L * Ly)
            path[cell] += h_e
            w -= dw
    return flux, path, leak


@pytest.mark.parametrize("Ly", [0.0, 0.4, 1.7])
def test_straight_network_gives_straight_lines(orc, Ly):
    prob = inputs.Problem(6, 5, 0.5, np.tile(_T[:6], 5), np.tile(_C[:6], 5), 2, 1, 2, 2, Ly=Ly)
    n = 1200
    w = straight_network(11 if Ly > 0 else 10)
    got = orc.transport_composed(prob, 9, np.arange(n), orc.stage2_generative(w, 1))
    flux, path, leak = _straight_lines(orc, prob, 9, n)
    np.testing.assert_allclose(got["flux"], flux, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(got["path"], path, rtol=1e-9, atol=1e-12)
    assert got["leak"].sum() == pytest.approx(leak, rel=1e-9)
    assert got["rejected_n"].sum() == 0 and not got["at_risk"]
