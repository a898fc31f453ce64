"""Pins for the oracle's cell-to-cell transport (paper section "Transport Algorithm", the
track-length estimator of eqs. 5-7, and the convergence metric of eq. 12)."""
import math

import numpy as np
import pytest

from paper_2512_13965_amd import inputs

NT = 8


def test_weight_balance_per_run(orc):
    # P6: every unit of source weight leaks, is absorbed, or is cut off
    prob = inputs.checkerboard_problem(8, src=2)
    n = 4000
    r = orc.transport(prob, seed=1, h_begin=0, h_end=n, nthreads=NT)
    total = r["leak"] + r["absorbed"].sum() + r["cutoff"]
    assert abs(total - n) < 1e-9 * n
    assert r["cutoff"] < 1e-6 * n * 10


def test_reflecting_box_flux_equals_source_over_sigma_a(orc):
    # P7: homogeneous reflecting box, uniform isotropic source of N particles:
    # all weight is absorbed (up to the cutoff), sum_i sigma_a phi_i V = N, and by symmetry
    # E[phi_i] = N / (sigma_a V n_cells) in every cell.
    tau, c, L = 2.0, 0.8, 0.5
    prob = inputs.homogeneous_problem(6, tau, c, reflect=True, L=L)
    n = 20_000
    r = orc.transport(prob, seed=2, h_begin=0, h_end=n, nthreads=NT)
    sig_a = (1 - c) * tau / L
    V = L * L
    assert r["leak"] == 0.0
    assert abs(r["absorbed"].sum() + r["cutoff"] - n) < 1e-9 * n
    np.testing.assert_allclose((r["flux"] * sig_a * V).sum(), r["absorbed"].sum(), rtol=1e-12)
    phi_exp = n / (sig_a * V * prob.n_cells)
    # per-cell fluctuations: compare with independent repeats
    reps = [orc.transport(prob, seed=10 + k, h_begin=0, h_end=n, nthreads=NT)["flux"]
            for k in range(4)]
    reps = np.array(reps + [r["flux"]])
    m = reps.mean(0)
    se = reps.std(0, ddof=1) / math.sqrt(reps.shape[0])
    z = np.abs(m - phi_exp) / np.maximum(se, 1e-12)
    assert np.median(z) < 2.0
    assert abs(m.mean() - phi_exp) / phi_exp < 2e-3


def test_vacuum_thin_grid_leaks_everything(orc):
    prob = inputs.homogeneous_problem(4, 1e-9, 0.0, reflect=False)
    n = 2000
    r = orc.transport(prob, seed=3, h_begin=0, h_end=n, nthreads=NT)
    assert abs(r["leak"] - n) < 1e-6 * n
    # flux of a pure streamer: track length per unit volume; total track length of
    # isotropic chords from uniform points in a 4x4 square
    assert r["flux"].sum() > 0


def test_histories_are_independent_of_chunking(orc):
    prob = inputs.checkerboard_problem(8, src=2)
    a = orc.transport(prob, seed=4, h_begin=0, h_end=600, nthreads=1)
    b = orc.transport(prob, seed=4, h_begin=0, h_end=250, nthreads=3)
    c = orc.transport(prob, seed=4, h_begin=250, h_end=600, nthreads=2)
    np.testing.assert_allclose(a["flux"], b["flux"] + c["flux"], rtol=1e-12, atol=1e-15)
    assert a["events"] == b["events"] + c["events"]


@pytest.mark.slow
def test_eq12_statistical_error_decays_as_inverse_sqrt_n(orc):
    # eq. 12: cell-averaged standard deviation over K = 5 runs, slope -1/2 in log-log
    prob = inputs.checkerboard_problem(8, src=2)
    Ns = [1000, 4000, 16000]
    sig = []
    for N in Ns:
        runs = np.array([orc.transport(prob, seed=100 + k, h_begin=0, h_end=N, nthreads=NT)["flux"]
                         / N for k in range(5)])
        sig.append(np.mean(runs.std(0, ddof=1)))
    slope = np.polyfit(np.log(Ns), np.log(sig), 1)[0]
    assert abs(slope + 0.5) < 0.1


def _global_walk_flux(prob, n, seed, paths=None):
    """Brute-force reference: one continuous random walk per history in global coordinates
    over the whole grid (no per-cell canonical frames), flights from the local sigma_s,
    continuous absorption per segment, track-length tally per segment.  Pure Python.  With
    `paths` (a dict), also the per-cell path tallies of every cell visit (from entering a cell
    to leaving it): paths["wpath"] += w at entry * track length in the cell, paths["path"] +=
    track length, paths["visits"] += 1."""
    g = np.random.default_rng(seed)
    L = prob.L
    Ly = prob.Ly if prob.Ly > 0 else L

    def direction():
        # isotropic: on the circle (flatland) or on the sphere, projected (XY geometry)
        ph = 2 * math.pi * g.random()
        st = math.sqrt(1.0 - (2.0 * g.random() - 1.0) ** 2) if prob.xy else 1.0
        return st * math.cos(ph), st * math.sin(ph)
    flux = np.zeros(prob.n_cells)
    if paths is not None:
        for k in ("wpath", "path", "visits"):
            paths[k] = np.zeros(prob.n_cells)
    for _ in range(n):
        k = g.integers(prob.src_nx * prob.src_ny)
        ci = prob.src_x0 + k % prob.src_nx
        cj = prob.src_y0 + k // prob.src_nx
        x = (ci + g.random()) * L
        y = (cj + g.random()) * Ly
        u, v = direction()
        w = 1.0
        d_s = None
        w_in, l_in = 1.0, 0.0
        while True:
            cell = cj * prob.nx + ci
            sig_t = prob.tau[cell] / L
            sig_s = prob.c[cell] * sig_t
            sig_a = sig_t - sig_s
            if d_s is None:
                d_s = -math.log(1.0 - g.random()) / sig_s if sig_s > 0 else math.inf
            tx = ((ci + 1) * L - x) / u if u > 0 else ((ci * L - x) / u if u < 0 else math.inf)
            ty = ((cj + 1) * Ly - y) / v if v > 0 else ((cj * Ly - y) / v if v < 0 else math.inf)
            db = min(tx, ty)
            seg = min(db, d_s)
            dw = w * (-math.expm1(-sig_a * seg))
            flux[cell] += (dw / sig_a if sig_a > 0 else w * seg) / (L * Ly)
            w -= dw
            x += seg * u
            y += seg * v
            l_in += seg
            if d_s < db:
                u, v = direction()
                d_s = None
                continue
            d_s = None         # exponential flights are memoryless: redraw in the next cell
            if paths is not None:
                paths["wpath"][cell] += w_in * l_in
                paths["path"][cell] += l_in
                paths["visits"][cell] += 1.0
            w_in, l_in = w, 0.0
            if tx <= ty:
                ci += 1 if u > 0 else -1
            else:
                cj += 1 if v > 0 else -1
            if ci < 0 or cj < 0 or ci >= prob.nx or cj >= prob.ny:
                break
            if w < prob.w_min:
                break
    return flux


@pytest.mark.parametrize("Ly,xy", [(0.0, False), (0.35, False), (1.6, False), (0.0, True), (0.5, True)])
def test_cell_to_cell_transport_matches_global_walk(orc, Ly, xy):
    # the per-cell canonical rotation (stage 1), face decoding and neighbour move (stage 4)
    # must reproduce a plain global random walk over the same heterogeneous grid, for square
    # cells and for rectangles of either orientation (canonical frames with A = W / H and H / W),
    # in flatland and in XY geometry (three-dimensional directions, projected)
    t = np.array([0.3, 2.0, 0.7, 1.5, 0.5, 3.0, 0.9, 0.2, 1.1])
    c = np.array([0.9, 0.5, 0.99, 0.7, 0.8, 0.95, 0.3, 1.0, 0.6])
    prob = inputs.Problem(3, 3, 0.7, t, c, 1, 1, 1, 1, Ly=Ly, xy=xy)
    n, runs = 3000, 5
    refp = [dict() for _ in range(runs)]
    ref = np.array([_global_walk_flux(prob, n, seed=s, paths=refp[s]) / n for s in range(runs)])
    orcs = [orc.transport(prob, seed=40 + s, h_begin=0, h_end=n, nthreads=NT) for s in range(runs)]
    got = np.array([o["flux"] / n for o in orcs])
    se = np.sqrt(ref.var(0, ddof=1) / runs + got.var(0, ddof=1) / runs)
    z = np.abs(ref.mean(0) - got.mean(0)) / np.maximum(se, 1e-12)
    assert z.max() < 5.0, z
    # the path tallies of every cell visit (the third stage's physical track length)
    for k in ("wpath", "path", "visits"):
        a = np.array([r[k] / n for r in refp])
        b = np.array([o[k] / n for o in orcs])
        se = np.sqrt(a.var(0, ddof=1) / runs + b.var(0, ddof=1) / runs)
        z = np.abs(a.mean(0) - b.mean(0)) / np.maximum(se, 1e-12)
        assert z.max() < 5.0, (k, z)


def test_visit_cap_ends_histories_that_would_never_end(orc):
    # a reflecting box without absorption keeps every history forever; with max_visits = M a
    # volumetric birth is transmitted in visits 0 .. M-1 and then cut off: cutoff = n exactly,
    # nothing absorbed or leaked, M transmissions per history
    n, M = 2_000, 50
    prob = inputs.homogeneous_problem(4, 1.0, 1.0, reflect=True)
    prob.max_visits = M
    o = orc.transport(prob, seed=3, h_begin=0, h_end=n, nthreads=4)
    assert o["cutoff"] == pytest.approx(n, rel=1e-12)
    assert o["leak"] == 0.0 and np.all(o["absorbed"] == 0.0)
    assert o["events"] == M * n
    # a larger cap gives each history more visits: the flux grows in proportion
    prob.max_visits = 2 * M
    o2 = orc.transport(prob, seed=3, h_begin=0, h_end=n, nthreads=4)
    assert o2["events"] == 2 * M * n
    assert 1.8 < o2["flux"].sum() / o["flux"].sum() < 2.2


def test_path_tally_invariants(orc):
    # with sigma_a = 0 the flux estimator of a visit is w_in * l / V, so flux * V equals the
    # weighted path tally; elsewhere dw / sigma_a <= w_in * l; weights never exceed 1, so the
    # unweighted path tally bounds the weighted one; every sampled transmission is one visit
    prob = inputs.checkerboard_problem(8, tau=(0.5, 3.0), c=(1.0, 0.7), src=2)
    n = 3000
    r = orc.transport(prob, seed=6, h_begin=0, h_end=n, nthreads=NT)
    V = prob.L ** 2
    pure = prob.c == 1.0
    np.testing.assert_allclose(r["flux"][pure] * V, r["wpath"][pure], rtol=1e-12)
    assert np.all(r["flux"][~pure] * V <= r["wpath"][~pure] * (1 + 1e-12))
    assert np.all(r["wpath"] <= r["path"] * (1 + 1e-12))
    assert r["visits"].sum() == r["events"]
    assert np.all(r["visits"] == np.round(r["visits"]))


def test_p3_mean_track_per_cell_visit(orc):
    # P3 (mean-chord invariance, per cell type): in a reflecting box of pure scatterers (any
    # per-cell thickness) a uniform isotropic field stays uniform and isotropic, so a cell is
    # entered uniformly along its faces with the cosine law and the mean track per entry is
    # pi A / P = pi L / 4, whatever the cell's thickness.  Histories are cut at visit M; two caps
    # M1 < M2 run the same random numbers for the first M1 visits, so the difference of the path
    # tallies holds exactly the visits M1 .. M2 - 1 (entries long after the birth leg).
    t = np.where((np.arange(4)[:, None] + np.arange(4)[None, :]) % 2 == 0, 0.5, 20.0).reshape(-1)
    L = 0.5
    prob = inputs.Problem(4, 4, L, t, np.ones(16), 0, 0, 4, 4, reflect=True)
    n = 6000
    out = {}
    for M in (16, 64):
        prob.max_visits = M
        out[M] = orc.transport(prob, seed=8, h_begin=0, h_end=n, nthreads=NT)
    dl = out[64]["path"] - out[16]["path"]
    dv = out[64]["visits"] - out[16]["visits"]
    assert dv.sum() == n * 48
    thin = t == 0.5
    for sel in (thin, ~thin):
        mean = dl[sel].sum() / dv[sel].sum()
        # per-visit tracks have a standard deviation below L; 4 sigma with room for the
        # correlation along a history
        tol = 4 * L * math.sqrt(4.0 / dv[sel].sum())
        assert abs(mean - math.pi * L / 4) < tol, (mean, math.pi * L / 4, tol)
    # the weighted tally equals the unweighted one (w = 1 throughout without absorption)
    np.testing.assert_allclose(out[64]["wpath"], out[64]["path"], rtol=1e-12)
