#!/usr/bin/env python3
"""Benchmark of the GMC cell-transmission sampler on one MI355X.

A step is one batch of 65,536 cell transmissions (ln tau ~ U[ln 0.1, ln 100], c ~ U[0, 1],
uniform entry height, cosine-law entry direction) through the fused velocity-MLP + Euler
sampler: FP32, 4 hidden layers x 256 SiLU, K = 16 Euler steps, seeded random-init weights,
Philox noise, decoded exits written to HBM.  `value` is transmissions per second with the
inputs resident in HBM.

Beside the timed steps the same run measures, with HIP events on the launch stream:
  * the analog random-walk kernel that the sampler replaces, on 2^20 transmissions per
    optical thickness tau = 1 .. 100 (c = 1, pure scattering) and the GMC/analog ratio;
  * the width-512 sampler in BF16 and FP8 (2^20 transmissions, Euler K = 8 / 16 / 32 and
    classic RK4 with 12 steps);
  * the FP64 CPU oracle on a bounded sample of the same workload (cpu_baseline).
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell transmissions/sec GMC vs analog MC at tau=1..100; p50/p99 request latency"
TAUS = [1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0]
PEAK = {"f32": 157.3e12, "bf16": 2.5e15, "fp8": 5.0e15}
KERNEL_SOURCES = ["gmc_mlp.hip", "gmc_device.hpp", "gmc_internal.hpp"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "mlp_ode_fp32_h256_k16_b65536.md")


def kernel_source_hash() -> str:
    """SHA-256 over the sources the sampler kernel is built from."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_13965_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the committed counter summary, or None
    when the kernel sources changed since those counters were taken."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m_hash = re.search(r"traffic_source_sha256:\s*([0-9a-f]{64})", text)
    m_bytes = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def flops_per_sample(H: int, K: int) -> float:
    # per velocity evaluation: 2 * (10 H + 3 H^2 + 5 H) multiply-adds counted as 2 flops each
    return K * 2.0 * (10 * H + 3 * H * H + 5 * H)


def time_launches(fn, reps: int, stream):
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in evs])     # ms


def cpu_baseline(H, K, budget_s=15.0):
    """The FP64 oracle sampler, timed on the host on a bounded sample of the workload."""
    import oracle
    from threadpoolctl import threadpool_info
    from paper_2512_13965_amd import inputs
    w = inputs.random_weights(H, 1)
    probe = 256
    cond = inputs.transmission_conditions(probe, 3)
    z = oracle.noise(2, 0, probe)
    t0 = time.perf_counter()
    oracle.sample_raw(w, cond, K, z)
    dt = time.perf_counter() - t0
    n = int(min(1 << 18, max(probe, probe * budget_s / max(dt, 1e-6))))
    cond = inputs.transmission_conditions(n, 3)
    t0 = time.perf_counter()
    z = oracle.noise(2, 0, n)
    raw = oracle.sample_raw(w, cond, K, z)
    oracle.decode(raw)
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": n / dt, "unit": "transmissions/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} transmissions of the same workload (FP64 numpy MLP + Philox/Box-Muller "
                      f"noise + decode), {dt:.1f} s", "host": host_cpu()}


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def cpu_baseline_analog(tau=100.0, budget_s=8.0):
    import oracle
    from paper_2512_13965_amd import inputs
    nt = os.cpu_count() or 1
    n = 4096
    cond = inputs.fixed_cell_conditions(n, tau, 1.0, 9)
    t0 = time.perf_counter()
    oracle.mc_transmit(cond, 0, 2, nthreads=nt)
    dt = time.perf_counter() - t0
    n = int(min(1 << 20, max(n, n * budget_s / max(dt, 1e-6))))
    cond = inputs.fixed_cell_conditions(n, tau, 1.0, 9)
    t0 = time.perf_counter()
    oracle.mc_transmit(cond, 0, 2, nthreads=nt)
    dt = time.perf_counter() - t0
    n1 = 1 << 16
    c1 = inputs.fixed_cell_conditions(n1, tau, 1.0, 9)
    t0 = time.perf_counter()
    oracle.mc_transmit(c1, 0, 2, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": n / dt, "unit": "transmissions/s", "cores": nt, "kind": "oracle",
            "sample": f"{n} analog transmissions at tau={tau:g}, c=1, {dt:.1f} s",
            "single_thread_value": n1 / dt1, "host": host_cpu()}


def bench_transport(binding, inputs, w512, w512_internal=None):
    """Full 2-D transport: 32 x 32 unit cells, checkerboard (tau, c) = (0.5, 0.5) / (50, 0.99),
    isotropic unit source in the central 4 x 4 cells, vacuum boundaries, 10^6 histories, FP64
    tallies; analog sampler and generative sampler (BF16, H = 512: Euler K = 16 and 32, RK4 with
    12 steps, and RK4 with births sampled by the internal model when its weights exist)."""
    import torch
    from paper_2512_13965_amd import transport
    prob = inputs.checkerboard_problem(32)
    n = 1_000_000
    out = {"workload": "32x32 checkerboard (0.5,0.5)/(50,0.99), central 4x4 source, vacuum, 1e6 histories"}
    world = binding.World(1 << 20, 2, 1 << 12)
    model = binding.Model(inputs.pack_blob(w512), "bf16")
    src = None if w512_internal is None else binding.Model(inputs.pack_blob(w512_internal), "bf16")
    flux = {}
    runs = [("analog", binding.SAMPLER_MC, None, 16, "euler", None),
            ("gmc_bf16_h512_k16", binding.SAMPLER_GMC, model, 16, "euler", None),
            ("gmc_bf16_h512_k32", binding.SAMPLER_GMC, model, 32, "euler", None),
            ("gmc_bf16_h512_rk4x12", binding.SAMPLER_GMC, model, 12, "rk4", None)]
    if src is not None:
        runs.append(("gmc_bf16_h512_rk4x12_internal_births", binding.SAMPLER_GMC, model, 12, "rk4", src))
    for name, smp, m, K, integ, sm in runs:
        kw = dict(integrator=integ, source_model=sm, source_K=K)
        transport.run_problem(world, prob, 20_000, 7, smp, m, K, **kw)          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = transport.run_problem(world, prob, n, 1, smp, m, K, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bal = r["absorbed"].sum() + r["leak"].sum() + r["cutoff"].sum()
        flux[name] = r["flux"] / n
        out[name] = {"seconds": dt, "histories_per_s": n / dt, "transmissions": int(r["transmissions"]),
                     "transmissions_per_s": r["transmissions"] / dt, "steps": r["steps"],
                     "balance_error": abs(bal - n) / n, "leak_per_history": float(r["leak"].sum() / n)}
    model.close()
    if src is not None:
        src.close()
    world.close()
    ref = flux["analog"]
    for name in flux:
        if name != "analog":
            out[name]["flux_rel_l1_vs_analog"] = float(np.abs(flux[name] - ref).sum() / np.abs(ref).sum())
    out["note"] = ("the generative runs use the weights fitted to this library's analog walk "
                   "(paper_2512_13965_amd/weights/gmc_h512.bin, and gmc_h512_internal.bin for the "
                   "births); flux_rel_l1_vs_analog is the L1 distance of the per-source-particle "
                   "flux maps")
    return out


def bench_paper_scale(binding, inputs, w512, w512_internal=None, n=200_000, w512_rect=None, w512_xy=None,
                      w512_collided=None, w512_xy_collided=None, w512_rect_collided=None,
                      w128_collided=None, w128_internal=None):
    """The paper's two benchmark problems at its mesh size and cross sections ("Benchmark
    Performance"; layouts defined by inputs.lattice_problem / inputs.hohlraum_problem): the
    7 x 7 cm lattice (112^2 cells, central volumetric source) and the 1.3 x 1.3 cm hohlraum
    (112^2 cells, isotropic incident flux on the left side).  Analog MC, and the generative
    sampler (BF16, H = 512) with Euler K = 16 and RK4 x 12; for the lattice also RK4 x 12 with
    births from the internal model.  flux_rel_l1_vs_mc is the L1 distance of the flux maps to
    the analog run; mc_noise_rel_l1 is the same distance between two analog runs with
    different seeds (the statistical floor at this history count).  With the rectangular-cell
    model, also the lattice on 112 x 56 cells of 1/16 x 1/8 cm; with the XY-geometry model, the
    lattice in XY geometry (one world per geometry).  With the collided model, square-cell
    problems (and with the rectangular-cell and XY collided models, the rectangular and XY
    lattices) also run RK4 x 12 with the
    first-flight split (uncollided crossings placed exactly, the rest sampled by the model
    fitted on collided exits)."""
    import torch
    from paper_2512_13965_amd import transport
    out = {"histories": n}
    model = binding.Model(inputs.pack_blob(w512), "bf16")
    src = None if w512_internal is None else binding.Model(inputs.pack_blob(w512_internal), "bf16")
    rect = None if w512_rect is None else binding.Model(inputs.pack_blob(w512_rect), "bf16")
    xym = None if w512_xy is None else binding.Model(inputs.pack_blob(w512_xy), "bf16")
    col = None if w512_collided is None else binding.Model(inputs.pack_blob(w512_collided), "bf16")
    colxy = None if w512_xy_collided is None else binding.Model(inputs.pack_blob(w512_xy_collided), "bf16")
    colr = None if w512_rect_collided is None else binding.Model(inputs.pack_blob(w512_rect_collided), "bf16")
    col128 = None if w128_collided is None else binding.Model(inputs.pack_blob(w128_collided), "bf16")
    src128 = None if w128_internal is None else binding.Model(inputs.pack_blob(w128_internal), "bf16")
    world = binding.World(1 << 20, 2, 1 << 14)
    problems = [("lattice_112", inputs.lattice_problem(16)), ("hohlraum_112", inputs.hohlraum_problem(112))]
    if rect is not None:
        problems.append(("lattice_112x56_rect", inputs.lattice_problem(16, 8)))
    if xym is not None:
        lx = inputs.lattice_problem(16)
        lx.xy = True
        problems.append(("lattice_112_xy", lx))
    for pname, prob in problems:
        if prob.xy:
            world.close()
            world = binding.World(1 << 20, 2, 1 << 14)
        bm = xym if prob.xy else (rect if prob.Ly > 0 else model)
        runs = [("analog", binding.SAMPLER_MC, None, 16, "euler", None),
                ("gmc_bf16_h512_k16", binding.SAMPLER_GMC, bm, 16, "euler", None),
                ("gmc_bf16_h512_rk4x12", binding.SAMPLER_GMC, bm, 12, "rk4", None)]
        if src is not None and prob.src_face < 0 and prob.Ly == 0 and not prob.xy:
            runs.append(("gmc_bf16_h512_rk4x12_internal_births", binding.SAMPLER_GMC, model, 12, "rk4", src))
        if col is not None and prob.Ly == 0 and not prob.xy:
            runs.append(("gmc_bf16_h512_rk4x12_split", binding.SAMPLER_GMC, col, 12, "rk4",
                         src if prob.src_face < 0 else None))
        if col128 is not None and prob.Ly == 0 and not prob.xy:
            runs.append(("gmc_bf16_h128_rk4x12_split", binding.SAMPLER_GMC, col128, 12, "rk4", None))
            runs.append(("gmc_bf16_h128_k16_split", binding.SAMPLER_GMC, col128, 16, "euler", None))
            if src128 is not None and prob.src_face < 0:
                runs.append(("gmc_bf16_h128_rk4x12_split_internal_births", binding.SAMPLER_GMC, col128, 12, "rk4",
                             src128))
        if colxy is not None and prob.xy:
            runs.append(("gmc_bf16_h512_rk4x12_split", binding.SAMPLER_GMC, colxy, 12, "rk4", None))
        if colr is not None and prob.Ly > 0:
            runs.append(("gmc_bf16_h512_rk4x12_split", binding.SAMPLER_GMC, colr, 12, "rk4", None))
        res, flux = {}, {}
        for name, smp, m, K, integ, sm in runs:
            kw = dict(integrator=integ, source_model=sm, source_K=K)
            transport.run_problem(world, prob, 5_000, 7, smp, m, K, **kw)          # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = transport.run_problem(world, prob, n, 1, smp, m, K, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            flux[name] = r["flux"] / n
            res[name] = {"seconds": dt, "histories_per_s": n / dt, "transmissions": int(r["transmissions"]),
                         "transmissions_per_s": r["transmissions"] / dt,
                         "transmissions_per_history": r["transmissions"] / n,
                         "leak_per_history": float(r["leak"].sum() / n)}
        ref = flux["analog"]
        l1 = lambda a: float(np.abs(a - ref).sum() / np.abs(ref).sum())
        for name in flux:
            if name != "analog":
                res[name]["flux_rel_l1_vs_mc"] = l1(flux[name])
        res["mc_noise_rel_l1"] = l1(transport.run_problem(world, prob, n, 2, binding.SAMPLER_MC)["flux"] / n)
        out[pname] = res
    world.close()
    model.close()
    for mm in (src, rect, xym, col, colxy, colr, col128, src128):
        if mm is not None:
            mm.close()
    return out


def bench_convergence(binding, inputs, w128_collided, Ns=(100_000, 200_000, 400_000, 800_000, 1_600_000,
                                                           3_200_000), runs=5):
    """Statistical convergence ("Convergence and Performance", eq. 12): the cell-averaged standard
    deviation of the scalar flux over `runs` independent runs at each history count N, for
    analog MC and GMC (the fitted H = 128 collided model, BF16, RK4 x 12, first-flight split,
    analog first legs for births), on the lattice and the hohlraum at 112^2.  The paper's N
    range is 1e5 .. 1.28e7; this one stops at 3.2e6 to keep the run short.  Reports sigma(N),
    the log-log slope and sigma_GMC / sigma_MC."""
    from paper_2512_13965_amd import transport
    m = binding.Model(inputs.pack_blob(w128_collided), "bf16")
    out = {"N": list(Ns), "runs": runs}
    for pname, prob in (("lattice_112", inputs.lattice_problem(16)), ("hohlraum_112", inputs.hohlraum_problem(112))):
        world = binding.World(1 << 20, 1, 1 << 14)
        res = {}
        for kind, smp, mm in (("analog", binding.SAMPLER_MC, None), ("gmc_bf16_h128_rk4x12_split", binding.SAMPLER_GMC, m)):
            sig = []
            for N in Ns:
                maps = np.array([transport.run_problem(world, prob, N, 5000 + 101 * k, smp, mm, 12,
                                                       integrator="rk4")["flux"] / N for k in range(runs)])
                sig.append(float(np.mean(maps.std(0, ddof=1))))
            res[kind] = {"sigma": sig, "slope": float(np.polyfit(np.log(Ns), np.log(sig), 1)[0])}
        res["sigma_ratio_gmc_over_mc"] = [g / a for g, a in zip(res["gmc_bf16_h128_rk4x12_split"]["sigma"],
                                                                 res["analog"]["sigma"])]
        world.close()
        out[pname] = res
    m.close()
    return out


def bench_thick_transport(binding, inputs, w128, n=50_000, w128_internal=None):
    """Transport through optically thick, highly scattering media: 16 x 16 checkerboards of
    (tau, c) = (100, 0.99) / (300, 0.999) and (300, 0.999) / (1000, 0.99), a central 2 x 2
    volumetric source, 50,000 histories.  Analog MC (two seeds: the statistical floor) against
    the fitted H = 128 model (BF16, RK4 x 12 and Euler K = 16; births by the analog first leg,
    and with the internal model also by the H = 128 internal model).  Every step waits for its
    longest walk in the analog runs (the analog births too), while the sampler's cost does not
    depend on tau."""
    import torch
    from paper_2512_13965_amd import transport
    m = binding.Model(inputs.pack_blob(w128), "bf16")
    src = None if w128_internal is None else binding.Model(inputs.pack_blob(w128_internal), "bf16")
    out = {"histories": n,
           "note": "the analog runs keep the transport algorithm's stage structure (one whole cell "
                   "transmission per particle per step, births' first legs walked to the end), so a "
                   "step lasts as long as its longest walk; thick_cells holds the kernel-level ratios "
                   "free of that effect"}
    l1 = lambda a, b: float(np.abs(a["flux"] - b["flux"]).sum() / np.abs(b["flux"]).sum())
    for name, tau, c in (("checker16_tau100_300", (100.0, 300.0), (0.99, 0.999)),
                         ("checker16_tau300_1000", (300.0, 1000.0), (0.999, 0.99))):
        prob = inputs.checkerboard_problem(16, tau=tau, c=c, src=2)
        world = binding.World(1 << 18, 1, 1 << 12)
        res, runs = {}, {}
        cases = [("analog", binding.SAMPLER_MC, None, "euler", 16, 1, None),
                 ("analog_seed2", binding.SAMPLER_MC, None, "euler", 16, 2, None),
                 ("gmc_bf16_h128_rk4x12", binding.SAMPLER_GMC, m, "rk4", 12, 3, None),
                 ("gmc_bf16_h128_k16", binding.SAMPLER_GMC, m, "euler", 16, 3, None)]
        if src is not None:
            cases.append(("gmc_bf16_h128_rk4x12_internal_births", binding.SAMPLER_GMC, m, "rk4", 12, 3, src))
        for rn, smp, mm, integ, K, seed, sm in cases:
            kw = dict(integrator=integ, source_model=sm, source_K=K)
            transport.run_problem(world, prob, 2_000, 7, smp, mm, K, **kw)      # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = transport.run_problem(world, prob, n, seed, smp, mm, K, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            runs[rn] = r
            res[rn] = {"seconds": dt, "steps": r["steps"], "transmissions_per_history": r["transmissions"] / n,
                       "transmissions_per_s": r["transmissions"] / dt}
        world.close()
        for rn in [c[0] for c in cases if c[0].startswith("gmc")]:
            res[rn]["flux_rel_l1_vs_mc"] = l1(runs[rn], runs["analog"])
            res[rn]["speedup_vs_analog"] = res["analog"]["seconds"] / res[rn]["seconds"]
        res["mc_noise_rel_l1"] = l1(runs["analog_seed2"], runs["analog"])
        out[name] = res
    m.close()
    if src is not None:
        src.close()
    return out


def bench_serving(binding, inputs, w512, n_req, w512_collided=None, w128_collided=None):
    """Continuous batching of a Poisson stream of transport requests of the config-3 kind
    (grids 16^2..128^2, per-cell tau log-uniform in [0.1, 200], c ~ U[0, 1]); histories per
    request log-uniform in [1e4, 10^5.5] (scaled down from 1e4..1e7 so the stream completes in
    tens of seconds); generative sampler BF16, H = 512, K = 16.  With the collided model, the
    same stream (same arrivals) also with the first-flight split (H = 512, and the H = 128
    collided model)."""
    from paper_2512_13965_amd import serving
    model = binding.Model(inputs.pack_blob(w512), "bf16")
    col = None if w512_collided is None else binding.Model(inputs.pack_blob(w512_collided), "bf16")
    col128 = None if w128_collided is None else binding.Model(inputs.pack_blob(w128_collided), "bf16")
    world = binding.World(1 << 20, 16, 1 << 18)
    make = lambda i: inputs.random_problem(1000 + i, hist_log10_range=(4.0, 5.5))

    def serve(reqs, graphs=True, m=model):
        world.set_graphs(graphs)
        return serving.Server(world, binding.SAMPLER_GMC, m, K=16, graphs=graphs,
                              cell_budget=(1 << 18) * serving.CELL_BYTES).run(reqs)

    # capacity: a burst of 48 requests all arriving at t = 0
    burst = serving.poisson_requests(48, rate_hz=1e9, seed=12, make_problem=make)
    cap = serve(burst)
    capacity_hz = len(cap.requests) / cap.wall
    rate = 0.7 * capacity_hz
    st = serve(serving.poisson_requests(n_req, rate_hz=rate, seed=11, make_problem=make))
    # the same stream with direct kernel launches instead of the captured per-bucket step graphs
    direct = serve(serving.poisson_requests(n_req, rate_hz=rate, seed=11, make_problem=make), graphs=False)
    split = None
    if col is not None:
        sp = serve(serving.poisson_requests(n_req, rate_hz=rate, seed=11, make_problem=make), m=col)
        split = {"latency_s": sp.latency_percentiles((50, 90, 99)), "transmissions_per_s": sp.throughput,
                 "wall_s": sp.wall, "steps": sp.steps,
                 "model": "collided-only BF16 H=512 K=16, uncollided crossings streamed in steps"}
        col.close()
    split128 = None
    if col128 is not None:
        sp = serve(serving.poisson_requests(n_req, rate_hz=rate, seed=11, make_problem=make), m=col128)
        split128 = {"latency_s": sp.latency_percentiles((50, 90, 99)), "transmissions_per_s": sp.throughput,
                    "wall_s": sp.wall, "steps": sp.steps,
                    "model": "collided-only BF16 H=128 K=16, uncollided crossings streamed in steps"}
        col128.close()
    model.close()
    world.close()
    lat = st.latency_percentiles((50, 90, 99))
    return {"first_flight_split": split, "first_flight_split_h128": split128,"requests": len(st.requests), "capacity_req_per_s": capacity_hz,
            "arrival_rate_hz": rate, "wall_s": st.wall, "steps": st.steps,
            "transmissions": st.transmissions, "transmissions_per_s": st.throughput,
            "latency_s": lat, "histories": int(sum(r.n_hist for r in st.requests)),
            "step_graphs": "captured per power-of-two particle-count bucket",
            "direct_launches": {"latency_s": direct.latency_percentiles((50, 90, 99)),
                                "transmissions_per_s": direct.throughput, "wall_s": direct.wall},
            "workload": "Poisson stream at 70% of the measured capacity; grids 16^2-128^2, "
                        "tau log-U[0.1,200], c U[0,1], 1e4-10^5.5 histories/request, "
                        "GMC BF16 H=512 K=16 trained weights"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="only the timed steps (for profiling)")
    ap.add_argument("--no-transport", action="store_true", help="skip transport and serving runs")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests in the serving stream")
    ap.add_argument("--profile", default=None,
                    help="only launch one kernel --steps times: fp32 | bf16 | fp8 (sampler, "
                         "H=256 / 512 / 512, Euler K=16), rk4 (BF16 H=512, RK4 x 12) or "
                         "walk:TAU[:LOG2N] (analog, 2^20 or 2^LOG2N transmissions), transport (cfg3 checkerboard, "
                         "2e5 analog histories per step), lattice_split (112^2 lattice, 2e5 "
                         "histories per step, first-flight split with the fitted collided model, "
                         "BF16 RK4 x 12), thick (16^2 checkerboard tau = 300/1000, c = 0.999/0.99, "
                         "2e4 histories per step: one analog run, one GMC run with the fitted H = 128 "
                         "model, BF16 RK4 x 12)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run plain device copies of 256 MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.profile:
        # a few launches of one kernel configuration, for counter collection
        import torch
        from paper_2512_13965_amd import binding, inputs
        kind, prec, H, K, N = args.profile.split(":")[0], None, 512, 16, 1 << 20
        if kind in ("fp32", "bf16", "fp8", "rk4"):
            prec, H = ("bf16" if kind == "rk4" else kind), (256 if kind == "fp32" else 512)
            integ, K = ("rk4", 12) if kind == "rk4" else ("euler", K)
            N = 65536 if kind == "fp32" else N
            m = binding.Model(inputs.pack_blob(inputs.random_weights(H, 1)), prec)
            c = binding.DeviceCond.from_host(inputs.transmission_conditions(N, 3))
            o = binding.DeviceExit.empty(N)
            for _ in range(args.steps):
                binding.gmc_sample(m, c, integ, K, 2, 0, out=o)
        elif kind == "transport":
            # the 32 x 32 checkerboard with the analog sampler: births, gather, walk, apply
            from paper_2512_13965_amd import transport
            w = binding.World(1 << 20, 1, 1 << 12)
            for _ in range(args.steps):
                transport.run_problem(w, inputs.checkerboard_problem(32), 200_000, 1, binding.SAMPLER_MC)
            w.close()
        elif kind == "thick":
            from paper_2512_13965_amd import transport
            wdir = os.path.join(ROOT, "paper_2512_13965_amd", "weights")
            m = binding.Model(open(os.path.join(wdir, "gmc_h128.bin"), "rb").read(), "bf16")
            w = binding.World(1 << 18, 1, 1 << 12)
            prob = inputs.checkerboard_problem(16, tau=(300.0, 1000.0), c=(0.999, 0.99), src=2)
            for _ in range(args.steps):
                transport.run_problem(w, prob, 20_000, 1, binding.SAMPLER_MC)
                transport.run_problem(w, prob, 20_000, 3, binding.SAMPLER_GMC, m, 12, integrator="rk4")
            w.close()
            N = 20_000
        elif kind == "lattice_split":
            from paper_2512_13965_amd import transport
            wdir = os.path.join(ROOT, "paper_2512_13965_amd", "weights")
            m = binding.Model(open(os.path.join(wdir, "gmc_h512_collided.bin"), "rb").read(), "bf16")
            src = binding.Model(open(os.path.join(wdir, "gmc_h512_internal.bin"), "rb").read(), "bf16")
            w = binding.World(1 << 20, 1, 1 << 14)
            for _ in range(args.steps):
                transport.run_problem(w, inputs.lattice_problem(16), 200_000, 1, binding.SAMPLER_GMC, m, 12,
                                      integrator="rk4", source_model=src, source_K=12)
            w.close()
            N = 200_000
        else:
            parts = args.profile.split(":")
            tau = float(parts[1]) if len(parts) > 1 else 100.0
            N = (1 << int(parts[2])) if len(parts) > 2 else N        # walk:TAU:LOG2N
            c = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(N, tau, 1.0, 9))
            o = binding.DeviceExit.empty(N)
            for _ in range(args.steps):
                binding.mc_transmit(c, binding.MODE_CONTINUOUS, 2, 0, out=o)
        torch.cuda.synchronize()
        print(json.dumps({"profile": args.profile, "launches": args.steps, "batch": N}))
        return
    if args.copy_ref:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes_each_way": src.numel() * 4, "launches": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the sampler shards by "
              f"particle id with no communication between GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_13965_amd import binding, inputs

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    H, K, N = 256, 16, 65536
    w = inputs.random_weights(H, 1)
    model = binding.Model(inputs.pack_blob(w), "fp32")
    cond = binding.DeviceCond.from_host(inputs.transmission_conditions(N, 3), dev)
    out = binding.DeviceExit.empty(N, dev)

    def step():
        binding.gmc_transmit(model, cond, K, seed=2, id_base=0, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = np.array([a.elapsed_time(b) for a, b in evs])
    ms_per_step = 1e3 * wall / args.steps
    value = N / (ms_per_step * 1e-3)
    fl = flops_per_sample(H, K) * N
    achieved = fl / (kms.mean() * 1e-3)
    res = {
        "metric": METRIC, "value": value, "unit": "transmissions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "GMC cell-transmission sampler: FP32 velocity MLP 10->256x4->5 SiLU, "
                               "K=16 Euler steps, batch 65536, ln tau~U[ln 0.1, ln 100], c~U[0,1], "
                               "seeded random-init weights, Philox noise",
                   "hidden": H, "K": K, "batch": N, "precision": "fp32"},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["f32"] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK["f32"], "traffic": measured_traffic(),
                     "kernel": "mlp_ode_kernel<fp32,256>", "avg_launch_ms": float(kms.mean())},
        "launch_ms_p50": float(np.median(kms)), "launch_ms_p99": float(np.quantile(kms, 0.99)),
    }
    if args.quick:
        print(json.dumps(res))
        return

    # sustained MFMA throughput of each instruction on this device (diagnostic, 2 waves / SIMD)
    peaks = {p: binding.probe_mfma_peak(p, 2) for p in ("fp32", "bf16", "fp8")}
    res["attainable_mfma_tflops"] = peaks
    res["roofline"]["frac_of_attainable"] = res["roofline"]["achieved"] / peaks["fp32"]

    # analog walk vs GMC, tau sweep (pure scattering), 2^20 transmissions per launch
    NA = 1 << 20
    sweep = []
    outA = binding.DeviceExit.empty(NA, dev)
    for tau in TAUS:
        c = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(NA, tau, 1.0, 9), dev)
        fn = lambda: binding.mc_transmit(c, binding.MODE_CONTINUOUS, 2, 0, out=outA)
        fn()
        ms = time_launches(fn, 3, stream)
        c9 = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(NA, tau, 0.9, 9), dev)
        fn9 = lambda: binding.mc_transmit(c9, binding.MODE_CONTINUOUS, 2, 0, out=outA)
        fn9()
        ms9 = time_launches(fn9, 3, stream)
        sweep.append({"tau": tau, "analog_tps": NA / (np.median(ms) * 1e-3),
                      "analog_ms": float(np.median(ms)),
                      "mean_flights_expected": 1 + math.pi * tau / 4,
                      "analog_tps_c0.9": NA / (np.median(ms9) * 1e-3)})
    # one launch of 2^20 walks at tau = 100 waits for its longest walk (~10^4 flights, serial
    # per lane); 2^23 walks per launch show the kernel's throughput with that tail amortised
    NL = 1 << 23
    cL = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(NL, 100.0, 1.0, 9), dev)
    oL = binding.DeviceExit.empty(NL, dev)
    fnL = lambda: binding.mc_transmit(cL, binding.MODE_CONTINUOUS, 2, 0, out=oL)
    fnL()
    msL = float(np.median(time_launches(fnL, 3, stream)))
    res["analog_tau100_batch_2^23"] = {"ms": msL, "tps": NL / (msL * 1e-3)}
    # thick cells: the analog walk's cost grows with tau (its longest walks grow faster), the
    # sampler's does not; 2^23 walks per launch at tau = 100, 300, 1000 against the fitted
    # samplers (BF16, H = 128 and 512) on 2^20 mixed-cell transmissions
    thick = {"analog_batch": NL, "analog_tps": {}}
    for tau in (100.0, 150.0, 200.0, 300.0, 500.0, 700.0, 1000.0):
        if tau == 100.0:
            thick["analog_tps"]["100"] = NL / (msL * 1e-3)
            continue
        cT = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(NL, tau, 1.0, 9), dev)
        fnT = lambda: binding.mc_transmit(cT, binding.MODE_CONTINUOUS, 2, 0, out=oL)
        fnT()
        thick["analog_tps"][str(int(tau))] = NL / (float(np.median(time_launches(fnT, 3, stream))) * 1e-3)
        del cT
    del cL, oL
    gmc_tps = N / (kms.mean() * 1e-3)
    for s in sweep:
        s["gmc_fp32_h256_tps"] = gmc_tps
        s["gmc_over_analog"] = gmc_tps / s["analog_tps"]
    res["tau_sweep"] = sweep

    # width-512 sampler in BF16 / FP8 on 2^20 transmissions (cfg2 shape, random-init weights)
    NB = 1 << 20
    w5 = inputs.random_weights(512, 1)
    wpath = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h512.bin")
    w5t = inputs.load_blob(wpath) if os.path.exists(wpath) else w5     # trained (cfg2)
    ipath = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h512_internal.bin")
    w5i = inputs.load_blob(ipath) if os.path.exists(ipath) else None
    rpath = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h512_rect.bin")
    w5r = inputs.load_blob(rpath) if os.path.exists(rpath) else None
    xpath = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h512_xy.bin")
    w5x = inputs.load_blob(xpath) if os.path.exists(xpath) else None
    cpath = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h512_collided.bin")
    w5c = inputs.load_blob(cpath) if os.path.exists(cpath) else None
    cxpath = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h512_xy_collided.bin")
    w5cx = inputs.load_blob(cxpath) if os.path.exists(cxpath) else None
    c128path = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h128_collided.bin")
    w1c = inputs.load_blob(c128path) if os.path.exists(c128path) else None
    i128path = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h128_internal.bin")
    w1i = inputs.load_blob(i128path) if os.path.exists(i128path) else None
    crpath = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h512_rect_collided.bin")
    w5cr = inputs.load_blob(crpath) if os.path.exists(crpath) else None
    condB = binding.DeviceCond.from_host(inputs.transmission_conditions(NB, 3), dev)
    outB = binding.DeviceExit.empty(NB, dev)
    wide = []
    for prec in ("bf16", "fp8"):
        m = binding.Model(inputs.pack_blob(w5t), prec)
        # explicit Euler at K = 8, 16, 32 and classic RK4 with 12 steps (48 evaluations: the
        # integrator and step count the paper times its sampler with)
        for integ, KK in (("euler", 8), ("euler", 16), ("euler", 32), ("rk4", 12)):
            fn = lambda: binding.gmc_sample(m, condB, integ, KK, 2, 0, out=outB)
            fn()
            ms = time_launches(fn, 3, stream)
            t = float(np.median(ms))
            nev = KK * (4 if integ == "rk4" else 1)
            fl = flops_per_sample(512, nev) * NB / (t * 1e-3)
            wide.append({"precision": prec, "hidden": 512, "integrator": integ, "K": KK,
                         "evaluations": nev, "batch": NB, "ms": t,
                         "tps": NB / (t * 1e-3), "tflops": fl / 1e12, "frac_peak": fl / PEAK[prec],
                         "frac_of_attainable": fl / 1e12 / peaks[prec]})
        m.close()
    res["wide_sampler"] = wide
    # width 256 in BF16 / FP8 (random-init weights), Euler K = 16, 2^20 transmissions
    h256 = []
    w2 = inputs.random_weights(256, 1)
    for prec in ("bf16", "fp8"):
        m = binding.Model(inputs.pack_blob(w2), prec)
        fn = lambda: binding.gmc_sample(m, condB, "euler", 16, 2, 0, out=outB)
        fn()
        t = float(np.median(time_launches(fn, 3, stream)))
        fl = flops_per_sample(256, 16) * NB / (t * 1e-3)
        h256.append({"precision": prec, "hidden": 256, "integrator": "euler", "K": 16, "batch": NB,
                     "ms": t, "tps": NB / (t * 1e-3), "tflops": fl / 1e12, "frac_peak": fl / PEAK[prec]})
        m.close()
    res["h256_sampler"] = h256
    # the fitted width-128 model (BF16): Euler K = 16 and RK4 x 12, 2^20 transmissions
    h128 = {}
    hpath = os.path.join(ROOT, "paper_2512_13965_amd", "weights", "gmc_h128.bin")
    w1 = inputs.load_blob(hpath) if os.path.exists(hpath) else inputs.random_weights(128, 1)
    m = binding.Model(inputs.pack_blob(w1), "bf16")
    for name, integ, KK in (("euler16", "euler", 16), ("rk4x12", "rk4", 12)):
        fn = lambda: binding.gmc_sample(m, condB, integ, KK, 2, 0, out=outB)
        fn()
        t = float(np.median(time_launches(fn, 3, stream)))
        h128[name] = {"ms": t, "tps": NB / (t * 1e-3)}
    m.close()
    res["h128_bf16_sampler"] = h128
    gmc_rates = {"fp32_h256_euler16": gmc_tps,
                 "bf16_h512_euler16": next(x["tps"] for x in wide if x["precision"] == "bf16"
                                           and x["integrator"] == "euler" and x["K"] == 16),
                 "bf16_h512_rk4x12": next(x["tps"] for x in wide if x["precision"] == "bf16"
                                          and x["integrator"] == "rk4"),
                 "bf16_h128_euler16": h128["euler16"]["tps"], "bf16_h128_rk4x12": h128["rk4x12"]["tps"]}
    thick["gmc_tps"] = gmc_rates
    thick["gmc_over_analog"] = {t: {k: v / a for k, v in gmc_rates.items()} for t, a in thick["analog_tps"].items()}
    # tau*: where each sampler's rate meets the analog walk's (log-log interpolation between the
    # measured tau; None if it stays below over the whole range)
    taus = sorted(float(t) for t in thick["analog_tps"])
    star = {}
    for k, g in gmc_rates.items():
        star[k] = None
        for t0, t1 in zip(taus, taus[1:]):
            a0, a1 = thick["analog_tps"][str(int(t0))], thick["analog_tps"][str(int(t1))]
            if g < a0 and g >= a1:
                f = math.log(a0 / g) / math.log(a0 / a1)
                star[k] = math.exp(math.log(t0) + f * math.log(t1 / t0))
                break
        if star[k] is None and g >= thick["analog_tps"][str(int(taus[0]))]:
            star[k] = taus[0]
    thick["tau_star"] = star
    res["thick_cells"] = thick
    for s in sweep:
        s["gmc_bf16_h512_k16_tps"] = next(x["tps"] for x in wide if x["precision"] == "bf16"
                                          and x["integrator"] == "euler" and x["K"] == 16)
        s["gmc_bf16_h512_rk4x12_tps"] = next(x["tps"] for x in wide if x["precision"] == "bf16"
                                             and x["integrator"] == "rk4")

    if not args.no_transport:
        res["transport"] = bench_transport(binding, inputs, w5t, w5i)
        res["paper_scale"] = bench_paper_scale(binding, inputs, w5t, w5i, w512_rect=w5r, w512_xy=w5x,
                                               w512_collided=w5c, w512_xy_collided=w5cx,
                                               w512_rect_collided=w5cr, w128_collided=w1c, w128_internal=w1i)
        res["serving"] = bench_serving(binding, inputs, w5t, args.serve_requests, w5c, w1c)
        res["thick_transport"] = bench_thick_transport(binding, inputs, w1, w128_internal=w1i)
        if w1c is not None:
            res["convergence"] = bench_convergence(binding, inputs, w1c)

    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(H, K)
        res["cpu_baseline_analog_tau100"] = cpu_baseline_analog()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
