#!/usr/bin/env python3
"""Benchmark of the GMC cell-transmission sampler on one MI355X.

A step is one launch of the generative sampler over a batch of 2^20 cell transmissions
(ln tau ~ U[ln 0.1, ln 100], c ~ U[0, 1], uniform entry height, cosine-law entry direction):
the velocity MLP 10 -> 512 x4 -> 5 (SiLU) with the fitted weights, BF16 operands and FP32
accumulation, K = 16 explicit Euler steps, Philox noise, decoded exit records written to HBM.
`value` is transmissions per second with the inputs resident in HBM.

The same run also measures, with HIP events on the launch stream:
  * the analog random walk that the sampler replaces, at tau = 1 .. 100 (c = 1) with 2^23
    walks per launch (throughput-bound), 2^20 at tau = 100 (tail-bound), and at tau = 150 ..
    1000 for the crossover thickness tau*;
  * the sampler's other precisions and integrators (FP8, K = 8 / 32, RK4 x 12) and the FP32
    H = 256 sampler on 65,536 transmissions;
  * a Poisson stream of transport requests (grids 16^2 .. 128^2, per-cell tau log-uniform in
    [0.1, 200], c ~ U[0, 1], 1e4 .. 1e7 histories each) served with continuous batching, p50 and
    p99 latency;
  * the FP64 CPU oracle on a bounded sample of the headline workload (cpu_baseline).

The last stdout line is one compact JSON record; the full results go to --detail (a JSON file).
`--study NAME` runs one of the longer studies instead (eq. 12 convergence on the 32 x 32
checkerboard, whole transport runs, the 112^2 benchmark layouts, thick media, the residual
network with adaptive modulation against the plain MLP).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
WDIR = os.path.join(ROOT, "paper_2512_13965_amd", "weights")

METRIC = "cell transmissions/sec GMC vs analog MC at tau=1..100; p50/p99 request latency"
TAUS = [1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0]
THICK_TAUS = [150.0, 200.0, 300.0, 500.0, 700.0, 1000.0]
PEAK = {"f32": 157.3e12, "bf16": 2.5e15, "fp8": 5.0e15}
HEAD_H, HEAD_K, HEAD_N = 512, 16, 1 << 20
KERNEL_SOURCES = ["gmc_mlp.hip", "gmc_mma.hpp", "gmc_device.hpp", "gmc_internal.hpp"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "mlp_ode_bf16_h512_k16_b1048576.md")


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


def flops_per_sample(H: int, evals: int) -> float:
    """Algorithmic FLOP of `evals` velocity evaluations of the 10 -> H x4 -> 5 network
    (multiply-adds counted as 2)."""
    return evals * 2.0 * (10 * H + 3 * H * H + 5 * H)


def algorithmic_bytes(N: int, weight_bytes: int) -> float:
    """Algorithmic HBM bytes of one sampler launch: 16 B of condition in and 20 B of exit
    record out per transmission, plus the weights once."""
    return 36.0 * N + weight_bytes


def time_launches(fn, reps: int, stream):
    """HIP-event durations (ms) of `reps` calls of fn, recorded on the launch stream."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in evs])


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


def fitted(name: str):
    from paper_2512_13965_amd import inputs
    p = os.path.join(WDIR, name)
    return inputs.load_blob(p) if os.path.exists(p) else None


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------------------------------
# CPU baselines (the FP64 oracle as it stands)
# ------------------------------------------------------------------------------------------

def cpu_baseline(w, K, budget_s=20.0):
    """The FP64 oracle sampler (numpy MLP, Philox + Box-Muller noise, decode) on a bounded
    sample of the headline workload, timed on the host."""
    import oracle
    from threadpoolctl import threadpool_info
    from paper_2512_13965_amd import inputs
    probe = 2048
    cond = inputs.transmission_conditions(probe, 3)
    t0 = time.perf_counter()
    oracle.sample_raw(w, cond, K, oracle.noise(2, 0, probe))
    dt = time.perf_counter() - t0
    n = int(min(1 << 18, max(probe, probe * budget_s / max(dt, 1e-6))))
    cond = inputs.transmission_conditions(n, 3)
    t0 = time.perf_counter()
    raw = oracle.sample_raw(w, cond, K, oracle.noise(2, 0, n))
    oracle.decode(raw)
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": n / dt, "unit": "transmissions/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {n} transmissions of the headline batch (FP64 MLP H={w.hidden}, "
                      f"K={K} Euler, noise, decode), {dt:.1f} s", "host": host_cpu()["model"]}


def cpu_baseline_analog(tau=100.0, budget_s=8.0):
    import oracle
    from paper_2512_13965_amd import inputs
    nt = os.cpu_count() or 1
    n = 4096
    cond = inputs.fixed_cell_conditions(n, tau, 1.0, 9)
    t0 = time.perf_counter()
    oracle.mc_transmit(cond, 0, 2, nthreads=nt)
    dt = time.perf_counter() - t0
    n = int(min(1 << 21, max(n, n * budget_s / max(dt, 1e-6))))
    cond = inputs.fixed_cell_conditions(n, tau, 1.0, 9)
    t0 = time.perf_counter()
    oracle.mc_transmit(cond, 0, 2, nthreads=nt)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "transmissions/s", "cores": nt, "kind": "oracle",
            "sample": f"{n} analog transmissions at tau={tau:g}, c=1, {dt:.1f} s"}


# ------------------------------------------------------------------------------------------
# GPU measurements beside the headline
# ------------------------------------------------------------------------------------------

def bench_analog(binding, inputs, dev, stream, reps=3):
    """Analog walk (mode C, c = 1 and 0.9) at 2^23 walks per launch for tau = 1 .. 100 and
    150 .. 1000, and at 2^20 for tau = 100."""
    NL, NS = 1 << 23, 1 << 20
    out = {"batch": NL, "tps": {}, "tps_c0.9": {}}
    oL = binding.DeviceExit.empty(NL, dev)
    for tau in TAUS + THICK_TAUS:
        for c, key in ((1.0, "tps"), (0.9, "tps_c0.9")):
            if c != 1.0 and tau > 100:
                continue
            cc = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(NL, tau, c, 9), dev)
            fn = lambda: binding.mc_transmit(cc, binding.MODE_CONTINUOUS, 2, 0, out=oL)
            fn()
            out[key][str(int(tau))] = NL / (float(np.median(time_launches(fn, reps, stream))) * 1e-3)
            del cc
        log(f"analog tau={tau:g}: {out['tps'][str(int(tau))]:.3e} /s")
    del oL
    cS = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(NS, 100.0, 1.0, 9), dev)
    oS = binding.DeviceExit.empty(NS, dev)
    fn = lambda: binding.mc_transmit(cS, binding.MODE_CONTINUOUS, 2, 0, out=oS)
    fn()
    out["tps_tau100_batch_2^20"] = NS / (float(np.median(time_launches(fn, reps, stream))) * 1e-3)
    return out


def tau_star(rate: float, analog_tps: dict):
    """Thickness where a sampler's rate meets the analog walk's (log-log interpolation between
    the measured tau); None if the sampler stays below over the whole range."""
    taus = sorted(float(t) for t in analog_tps)
    a = lambda t: analog_tps[str(int(t))]
    if rate >= a(taus[0]):
        return taus[0]
    for t0, t1 in zip(taus, taus[1:]):
        if a(t0) > rate >= a(t1):
            f = math.log(a(t0) / rate) / math.log(a(t0) / a(t1))
            return math.exp(math.log(t0) + f * math.log(t1 / t0))
    return None


def bench_samplers(binding, inputs, dev, stream, w512, reps=3):
    """The width-512 sampler in BF16 and FP8 (Euler K = 8, 16, 32; RK4 x 12), the width-512
    residual network with adaptive modulation (BF16; Euler K = 16, RK4 x 12), the fitted
    width-128 model, and the FP32 H = 256 sampler on 65,536 transmissions (random-init)."""
    NB = 1 << 20
    cond = binding.DeviceCond.from_host(inputs.transmission_conditions(NB, 3), dev)
    out_b = binding.DeviceExit.empty(NB, dev)
    rows = []
    for prec in ("bf16", "fp8"):
        m = binding.Model(inputs.pack_blob(w512), prec)
        for integ, KK in (("euler", 8), ("euler", 16), ("euler", 32), ("rk4", 12)):
            fn = lambda: binding.gmc_sample(m, cond, integ, KK, 2, 0, out=out_b)
            fn()
            t = float(np.median(time_launches(fn, reps, stream)))
            nev = KK * (4 if integ == "rk4" else 1)
            fl = flops_per_sample(512, nev) * NB / (t * 1e-3)
            rows.append({"precision": prec, "hidden": 512, "integrator": integ, "K": KK, "batch": NB,
                         "ms": t, "tps": NB / (t * 1e-3), "frac_peak": fl / PEAK[prec]})
        m.close()
    wf = fitted("gmc_film_h512.bin")
    wf = inputs.random_film_weights(512, 1) if wf is None else wf
    m = binding.Model(inputs.pack_blob(wf), "bf16")
    for integ, KK in (("euler", 16), ("rk4", 12)):
        fn = lambda: binding.gmc_sample(m, cond, integ, KK, 2, 0, out=out_b)
        fn()
        t = float(np.median(time_launches(fn, reps, stream)))
        fl = film_flops_per_sample(512, KK * (4 if integ == "rk4" else 1)) * NB / (t * 1e-3)
        rows.append({"precision": "bf16", "hidden": 512, "net": "residual, adaptive modulation",
                     "integrator": integ, "K": KK, "batch": NB, "ms": t, "tps": NB / (t * 1e-3),
                     "frac_peak": fl / PEAK["bf16"]})
    m.close()
    w128 = fitted("gmc_h128.bin")
    if w128 is not None:
        m = binding.Model(inputs.pack_blob(w128), "bf16")
        for integ, KK in (("euler", 16), ("rk4", 12)):
            fn = lambda: binding.gmc_sample(m, cond, integ, KK, 2, 0, out=out_b)
            fn()
            t = float(np.median(time_launches(fn, reps, stream)))
            ev = KK * (4 if integ == "rk4" else 1)
            rows.append({"precision": "bf16", "hidden": 128, "integrator": integ, "K": KK, "batch": NB,
                         "ms": t, "tps": NB / (t * 1e-3),
                         "frac_peak": flops_per_sample(128, ev) * NB / (t * 1e-3) / PEAK["bf16"]})
        m.close()
    N1 = 65536
    m = binding.Model(inputs.pack_blob(inputs.random_weights(256, 1)), "fp32")
    c1 = binding.DeviceCond.from_host(inputs.transmission_conditions(N1, 3), dev)
    o1 = binding.DeviceExit.empty(N1, dev)
    fn = lambda: binding.gmc_transmit(m, c1, 16, 2, 0, out=o1)
    fn()
    t = float(np.median(time_launches(fn, 5, stream)))
    rows.append({"precision": "fp32", "hidden": 256, "integrator": "euler", "K": 16, "batch": N1, "ms": t,
                 "tps": N1 / (t * 1e-3), "frac_peak": flops_per_sample(256, 16) * N1 / (t * 1e-3) / PEAK["f32"],
                 "weights": "random-init (seed 1)"})
    m.close()
    return rows


def bench_serving(binding, inputs, w512, n_req, hist_log10=(4.0, 7.0), load=0.7, rate_hz=None,
                  label="GMC BF16 H=512 K=16 fitted weights"):
    """Continuous batching of a Poisson stream of transport requests of the 2-D transport kind
    (grids 16^2 .. 128^2, per-cell tau log-uniform in [0.1, 200], c ~ U[0, 1], central
    (side/8)^2 source, histories log-uniform in [10^a, 10^b]); generative sampler BF16,
    H = 512, K = 16, fitted weights; step graphs per particle-count bucket.  The arrival rate
    is `load` times the capacity measured on a burst of 24 requests all arriving at once, or
    `rate_hz` when given (the same arrivals for another model)."""
    from paper_2512_13965_amd import serving
    model = binding.Model(inputs.pack_blob(w512), "bf16")
    world = binding.World(1 << 20, 16, 1 << 18)
    make = lambda i: inputs.random_problem(1000 + i, hist_log10_range=hist_log10)

    def serve(reqs):
        return serving.Server(world, binding.SAMPLER_GMC, model, K=16, graphs=True,
                              cell_budget=(1 << 18) * serving.CELL_BYTES).run(reqs)

    burst = serving.poisson_requests(24, rate_hz=1e9, seed=12, make_problem=make)
    cap = serve(burst)
    capacity_hz = len(cap.requests) / cap.wall
    log(f"serving capacity {capacity_hz:.2f} req/s ({cap.wall:.1f} s burst)")
    rate = load * capacity_hz if rate_hz is None else rate_hz
    st = serve(serving.poisson_requests(n_req, rate_hz=rate, seed=11, make_problem=make))
    model.close()
    world.close()
    hist = np.array([r.n_hist for r in st.requests])
    lat = st.latency_percentiles((50, 90, 99))
    tot = {k: sum(float(r.tallies[k].sum()) for r in st.requests) for k in ("rejected_n", "rejected_w", "cutoff")}
    return {"requests": len(st.requests), "capacity_req_per_s": capacity_hz, "arrival_rate_hz": rate,
            "wall_s": st.wall, "steps": st.steps, "transmissions": st.transmissions,
            "transmissions_per_s": st.throughput, "latency_s": lat,
            **sampler_health({"transmissions": st.transmissions, **tot}, int(hist.sum())),
            "histories": {"total": int(hist.sum()), "min": int(hist.min()), "max": int(hist.max())},
            "workload": f"Poisson stream at {load:.0%} of the measured capacity; grids 16^2-128^2, "
                        f"tau log-U[0.1,200], c U[0,1], 10^{hist_log10[0]:g}-10^{hist_log10[1]:g} "
                        f"histories/request; {label}; step graphs"}


# ------------------------------------------------------------------------------------------
# longer studies (--study)
# ------------------------------------------------------------------------------------------

def sampler_health(r: dict, n: int) -> dict:
    """Rejected generative samples in one transport run (decoded exits outside the cell, turned
    into cutoff weight): their share of the transmissions, the weight they removed per history,
    and the whole cutoff weight per history."""
    tx = max(int(r["transmissions"]), 1)
    return {"rejected_fraction": float(np.sum(r["rejected_n"]) / tx),
            "rejected_weight_per_history": float(np.sum(r["rejected_w"]) / n),
            "cutoff_per_history": float(np.sum(r["cutoff"]) / n)}


def study_serving(binding, inputs, w512, n_req=200):
    """The bench's serving stream served twice with the same arrivals: with the plain boundary
    model, and with the model fitted on collided crossings, whose steps run the first-flight
    split (uncollided crossings streamed inside the step); BF16, H = 512, K = 16."""
    out = {"plain": bench_serving(binding, inputs, w512, n_req)}
    wc = fitted("gmc_h512_collided.bin")
    if wc is not None:
        out["collided_split"] = bench_serving(binding, inputs, wc, n_req,
                                              rate_hz=out["plain"]["arrival_rate_hz"],
                                              label="GMC BF16 H=512 K=16 collided model, first-flight split")
    return out


def study_convergence(binding, inputs, w512, Ns=None, runs=5):
    """Statistical convergence (paper "Convergence and Performance", eq. 12) on the 32 x 32
    checkerboard ((tau, c) = (0.5, 0.5) / (50, 0.99), central 4 x 4 source, vacuum): the
    cell-averaged standard deviation of the flux over `runs` independent runs at each history
    count N = 1e5 .. 1.28e7, analog MC against GMC (BF16, H = 512, K = 16, fitted weights).
    Reports sigma(N), the log-log slope and sigma_GMC / sigma_MC."""
    from paper_2512_13965_amd import transport
    Ns = Ns or [100_000 * 2 ** k for k in range(8)]
    m = binding.Model(inputs.pack_blob(w512), "bf16")
    prob = inputs.checkerboard_problem(32)
    world = binding.World(1 << 20, 1, 1 << 12)
    out = {"problem": "32x32 checkerboard (0.5,0.5)/(50,0.99), central 4x4 source, vacuum", "N": Ns,
           "runs": runs}
    for kind, smp, mm in (("analog", binding.SAMPLER_MC, None), ("gmc_bf16_h512_k16", binding.SAMPLER_GMC, m)):
        sig, secs, health = [], [], []
        for N in Ns:
            t0 = time.perf_counter()
            rs = [transport.run_problem(world, prob, N, 5000 + 101 * k, smp, mm, 16) for k in range(runs)]
            secs.append(time.perf_counter() - t0)
            maps = np.array([r["flux"] / N for r in rs])
            sig.append(float(np.mean(maps.std(0, ddof=1))))
            health.append(sampler_health({k: sum(r[k] for r in rs) for k in ("transmissions", "rejected_n",
                                                                            "rejected_w", "cutoff")}, N * runs))
            log(f"convergence {kind} N={N}: sigma {sig[-1]:.3e} ({secs[-1]:.1f} s)")
        out[kind] = {"sigma": sig, "seconds": secs, "health": health,
                     "slope": float(np.polyfit(np.log(Ns), np.log(sig), 1)[0])}
    out["sigma_ratio_gmc_over_mc"] = [g / a for g, a in zip(out["gmc_bf16_h512_k16"]["sigma"], out["analog"]["sigma"])]
    world.close()
    m.close()
    return out


def study_transport(binding, inputs, w512, n=1_000_000):
    """Whole transport runs on the 32 x 32 checkerboard, 10^6 histories: analog sampler and
    the generative sampler (BF16, H = 512, fitted: Euler K = 16, RK4 x 12)."""
    import torch
    from paper_2512_13965_amd import transport
    prob = inputs.checkerboard_problem(32)
    out = {"workload": "32x32 checkerboard (0.5,0.5)/(50,0.99), central 4x4 source, vacuum, 1e6 histories"}
    world = binding.World(1 << 20, 2, 1 << 12)
    model = binding.Model(inputs.pack_blob(w512), "bf16")
    flux = {}
    for name, smp, m, K, integ in (("analog", binding.SAMPLER_MC, None, 16, "euler"),
                                   ("gmc_bf16_h512_k16", binding.SAMPLER_GMC, model, 16, "euler"),
                                   ("gmc_bf16_h512_rk4x12", binding.SAMPLER_GMC, model, 12, "rk4")):
        transport.run_problem(world, prob, 20_000, 7, smp, m, K, integrator=integ)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = transport.run_problem(world, prob, n, 1, smp, m, K, integrator=integ)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flux[name] = r["flux"] / n
        out[name] = {"seconds": dt, "histories_per_s": n / dt, "transmissions": int(r["transmissions"]),
                     "transmissions_per_s": r["transmissions"] / dt, "steps": r["steps"],
                     "leak_per_history": float(r["leak"].sum() / n), **sampler_health(r, n)}
        log(f"transport {name}: {dt:.2f} s")
    for name in flux:
        if name != "analog":
            out[name]["flux_rel_l1_vs_analog"] = float(np.abs(flux[name] - flux["analog"]).sum()
                                                       / np.abs(flux["analog"]).sum())
    model.close()
    world.close()
    return out


def study_paper_scale(binding, inputs, w512, n=200_000):
    """The paper's two benchmark problems at its mesh size and cross sections, on layouts
    defined here (lattice: 112^2 cells, central volumetric source; hohlraum: 112^2 cells,
    isotropic incident flux on the left side): analog MC against the generative sampler: at
    width 512 with RK4 x 12, every transmission sampled (BF16), the first-flight split with the
    collided model (BF16 and FP8 e4m3) and in the lattice the full method, births from the
    internal model as well (BF16 and FP8); at width 128 (BF16) the split and the full method
    with RK4 x 12 and with Euler K = 16."""
    import torch
    from paper_2512_13965_amd import transport
    opened = []

    def model(w, prec):
        if w is None:
            return None
        m = binding.Model(inputs.pack_blob(w), prec)
        opened.append(m)
        return m

    plain = model(w512, "bf16")
    wc, wi = fitted("gmc_h512_collided.bin"), fitted("gmc_h512_internal.bin")
    col = {p: model(wc, p) for p in ("bf16", "fp8")}
    src = {p: model(wi, p) for p in ("bf16", "fp8")}
    col128, src128 = model(fitted("gmc_h128_collided.bin"), "bf16"), model(fitted("gmc_h128_internal.bin"), "bf16")
    world = binding.World(1 << 20, 2, 1 << 14)
    out = {"histories": n}
    rk4, eul = ("rk4", 12), ("euler", 16)
    for pname, prob in (("lattice_112", inputs.lattice_problem(16)), ("hohlraum_112", inputs.hohlraum_problem(112))):
        lattice = pname.startswith("lattice")
        runs = [("analog", binding.SAMPLER_MC, None, rk4, {}),
                ("gmc_bf16_h512_rk4x12", binding.SAMPLER_GMC, plain, rk4, {})]
        for prec in ("bf16", "fp8"):
            if col[prec] is not None:
                runs.append((f"gmc_{prec}_h512_rk4x12_split", binding.SAMPLER_GMC, col[prec], rk4, {}))
            if lattice and col[prec] is not None and src[prec] is not None:
                runs.append((f"gmc_{prec}_h512_rk4x12_full", binding.SAMPLER_GMC, col[prec], rk4,
                             {"source_model": src[prec], "source_K": 12}))
        if col128 is not None:
            for integ, tag in ((rk4, "rk4x12"), (eul, "euler16")):
                runs.append((f"gmc_bf16_h128_{tag}_split", binding.SAMPLER_GMC, col128, integ, {}))
                if lattice and src128 is not None:
                    runs.append((f"gmc_bf16_h128_{tag}_full", binding.SAMPLER_GMC, col128, integ,
                                 {"source_model": src128, "source_K": integ[1]}))
        res, flux = {}, {}
        for name, smp, m, (integ, K), kw in runs:
            transport.run_problem(world, prob, 5_000, 7, smp, m, K, integrator=integ, streaming=64, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = transport.run_problem(world, prob, n, 1, smp, m, K, integrator=integ, streaming=64, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            flux[name] = r["flux"] / n
            res[name] = {"seconds": dt, "transmissions_per_s": r["transmissions"] / dt,
                         "leak_per_history": float(r["leak"].sum() / n), **sampler_health(r, n)}
            log(f"{pname} {name}: {dt:.3f} s")
        l1 = lambda a: float(np.abs(a - flux["analog"]).sum() / np.abs(flux["analog"]).sum())
        for name in flux:
            if name != "analog":
                res[name]["flux_rel_l1_vs_mc"] = l1(flux[name])
        res["mc_noise_rel_l1"] = l1(transport.run_problem(world, prob, n, 2, binding.SAMPLER_MC)["flux"] / n)
        out[pname] = res
    world.close()
    for m in opened:
        m.close()
    return out


def study_thick(binding, inputs, n=50_000):
    """Transport through optically thick, highly scattering media (16 x 16 checkerboards of
    (tau, c) = (100, 0.99) / (300, 0.999) and (300, 0.999) / (1000, 0.99), central 2 x 2
    source): analog MC against the fitted H = 128 model (BF16, RK4 x 12), with analog births and
    with births from the fitted H = 128 internal model."""
    import torch
    from paper_2512_13965_amd import transport
    w128, wi = fitted("gmc_h128.bin"), fitted("gmc_h128_internal.bin")
    m = binding.Model(inputs.pack_blob(w128), "bf16")
    src = None if wi is None else binding.Model(inputs.pack_blob(wi), "bf16")
    out = {"histories": n}
    for name, tau, c in (("checker16_tau100_300", (100.0, 300.0), (0.99, 0.999)),
                         ("checker16_tau300_1000", (300.0, 1000.0), (0.999, 0.99))):
        prob = inputs.checkerboard_problem(16, tau=tau, c=c, src=2)
        world = binding.World(1 << 18, 1, 1 << 12)
        res, runs = {}, {}
        cases = [("analog", binding.SAMPLER_MC, None, "euler", 16, 1, None),
                 ("analog_seed2", binding.SAMPLER_MC, None, "euler", 16, 2, None),
                 ("gmc_bf16_h128_rk4x12", binding.SAMPLER_GMC, m, "rk4", 12, 3, None)]
        if src is not None:
            cases.append(("gmc_bf16_h128_rk4x12_internal_births", binding.SAMPLER_GMC, m, "rk4", 12, 3, src))
        for rn, smp, mm, integ, K, seed, sm in cases:
            transport.run_problem(world, prob, 2_000, 7, smp, mm, K, integrator=integ, source_model=sm, source_K=K)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            runs[rn] = transport.run_problem(world, prob, n, seed, smp, mm, K, integrator=integ, source_model=sm,
                                             source_K=K)
            torch.cuda.synchronize()
            res[rn] = {"seconds": time.perf_counter() - t0, **sampler_health(runs[rn], n)}
            log(f"{name} {rn}: {res[rn]['seconds']:.2f} s")
        world.close()
        l1 = lambda a, b: float(np.abs(a["flux"] - b["flux"]).sum() / np.abs(b["flux"]).sum())
        for rn in runs:
            if rn.startswith("gmc"):
                res[rn]["flux_rel_l1_vs_mc"] = l1(runs[rn], runs["analog"])
                res[rn]["speedup_vs_analog"] = res["analog"]["seconds"] / res[rn]["seconds"]
        res["mc_noise_rel_l1"] = l1(runs["analog_seed2"], runs["analog"])
        out[name] = res
    m.close()
    if src is not None:
        src.close()
    return out


def film_flops_per_sample(H: int, evals: int, n_c: int = 4, E: int = 32, B: int = 3) -> float:
    """Algorithmic FLOP of `evals` evaluations of the residual network: input layer over
    13 + n_c features, embedding over 8 + n_c, per block the H x H map and the two E -> H
    modulation maps, output layer H -> 5 (multiply-adds counted as 2)."""
    return evals * 2.0 * (H * (13 + n_c) + E * (8 + n_c) + B * (H * H + 2 * H * E) + 5 * H)


def study_film(binding, inputs, w512, n=100_000):
    """The paper's network (residual blocks with adaptive modulation, learned time and
    condition embeddings; "Network Architecture and Inputs") against the plain MLP, both BF16,
    width 512, fitted on the same data: exit-law distances to the analog walk at fixed entry
    conditions (face TV, KS of position, exit cosine and ln path), the mean path at c = 1
    against pi / 4 (P3), whole transport on the 32 x 32 checkerboard (flux L1 to analog MC
    beside the analog-vs-analog floor) and the cost of a 2^20 launch, for Euler K = 16 and
    RK4 x 12."""
    import torch
    from scipy import stats
    from paper_2512_13965_amd import transport
    wf = fitted("gmc_film_h512.bin")
    if wf is None:
        return {"skipped": "no fitted residual network"}
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    models = {"mlp": binding.Model(inputs.pack_blob(w512), "bf16"),
              "film": binding.Model(inputs.pack_blob(wf), "bf16")}
    integs = (("euler", 16), ("rk4", 12))
    fix = lambda m, tau, c, y, s_: inputs.Conditions(*[np.full(m, np.float32(v)) for v in
                                                       (math.log(tau), c, y, s_)])
    out = {"exit_law": [], "mean_path": [], "cost": [], "transport": {}}
    for tau, c, y, s_ in ((1.0, 1.0, 0.5, 0.2), (10.0, 1.0, 0.3, 0.5), (100.0, 1.0, 0.5, -0.3),
                          (30.0, 0.95, 0.9, -0.8)):
        ref = binding.mc_transmit(binding.DeviceCond.from_host(fix(n, tau, c, y, s_), dev), binding.MODE_CONTINUOUS,
                                  17, 0).to_host()
        for name, m in models.items():
            for integ, K in integs:
                g = binding.gmc_sample(m, binding.DeviceCond.from_host(fix(n, tau, c, y, s_), dev), integ, K,
                                       5).to_host()
                fg = np.bincount(g["face"][g["face"] >= 0], minlength=4) / n
                fo = np.bincount(ref["face"], minlength=4) / n
                out["exit_law"].append({
                    "net": name, "integrator": integ, "K": K, "tau": tau, "c": c, "y_in": y, "sin_th": s_,
                    "face_tv": float(0.5 * np.abs(fg - fo).sum()),
                    "ks_pos": float(stats.ks_2samp(g["pos"] + g["face"], ref["pos"] + ref["face"]).statistic),
                    "ks_cos": float(stats.ks_2samp(g["dir_cos"], ref["dir_cos"]).statistic),
                    "ks_ln_path": float(stats.ks_2samp(np.log(g["path"]), np.log(ref["path"])).statistic)})
    for tau in (1.0, 10.0, 100.0):
        cond = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(200_000, tau, 1.0, 3), dev)
        for name, m in models.items():
            for integ, K in integs:
                g = binding.gmc_sample(m, cond, integ, K, 9).to_host()
                out["mean_path"].append({"net": name, "integrator": integ, "K": K, "tau": tau,
                                         "mean_path": float(g["path"].mean()), "pi_over_4": math.pi / 4})
    NB = 1 << 20
    cond = binding.DeviceCond.from_host(inputs.transmission_conditions(NB, 3), dev)
    ob = binding.DeviceExit.empty(NB, dev)
    for name, m in models.items():
        for integ, K in integs:
            fn = lambda: binding.gmc_sample(m, cond, integ, K, 2, 0, out=ob)
            fn()
            t = float(np.median(time_launches(fn, 5, stream)))
            ev = K * (4 if integ == "rk4" else 1)
            fl = (film_flops_per_sample(512, ev) if name == "film" else flops_per_sample(512, ev)) * NB
            out["cost"].append({"net": name, "integrator": integ, "K": K, "batch": NB, "ms": t,
                                "tps": NB / (t * 1e-3), "flop_per_launch": fl,
                                "frac_peak": fl / (t * 1e-3) / PEAK["bf16"]})
    prob = inputs.checkerboard_problem(32)
    world = binding.World(1 << 20, 1, 1 << 12)
    nh = 200_000
    flux = {"analog": transport.run_problem(world, prob, nh, 1, binding.SAMPLER_MC)["flux"] / nh,
            "analog_seed2": transport.run_problem(world, prob, nh, 2, binding.SAMPLER_MC)["flux"] / nh}
    for name, m in models.items():
        for integ, K in integs:
            r = transport.run_problem(world, prob, nh, 3, binding.SAMPLER_GMC, m, K, integrator=integ)
            flux[f"{name}_{integ}{K}"] = r["flux"] / nh
            out["transport"][f"{name}_{integ}{K}"] = sampler_health(r, nh)
    world.close()
    l1 = lambda a: float(np.abs(a - flux["analog"]).sum() / np.abs(flux["analog"]).sum())
    for k, v in flux.items():
        if k != "analog":
            out["transport"].setdefault(k, {})["flux_rel_l1_vs_analog"] = l1(v)
    out["transport"]["workload"] = f"32x32 checkerboard (0.5,0.5)/(50,0.99), central 4x4 source, {nh} histories"
    for m in models.values():
        m.close()
    return out


# ------------------------------------------------------------------------------------------

def profile_launches(args):
    """A few launches of one kernel configuration, for rocprofv3 traces and counters."""
    import torch
    from paper_2512_13965_amd import binding, inputs
    kind = args.profile.split(":")[0]
    if kind in ("bf16", "fp8", "rk4", "fp32"):
        prec = "bf16" if kind == "rk4" else kind
        integ, K = ("rk4", 12) if kind == "rk4" else ("euler", HEAD_K)
        H, N = (256, 65536) if kind == "fp32" else (HEAD_H, HEAD_N)
        w = inputs.random_weights(H, 1) if kind == "fp32" else fitted("gmc_h512.bin")
        m = binding.Model(inputs.pack_blob(w), prec)
        c = binding.DeviceCond.from_host(inputs.transmission_conditions(N, 3))
        o = binding.DeviceExit.empty(N)
        for s in range(args.steps):
            binding.gmc_sample(m, c, integ, K, 2, s * N, out=o)
    elif kind in ("h128", "h128_rk4"):
        # the fitted width-128 model (BF16), 2^20 transmissions
        integ, K = ("rk4", 12) if kind == "h128_rk4" else ("euler", HEAD_K)
        m = binding.Model(inputs.pack_blob(fitted("gmc_h128.bin")), "bf16")
        N = HEAD_N
        c = binding.DeviceCond.from_host(inputs.transmission_conditions(N, 3))
        o = binding.DeviceExit.empty(N)
        for s in range(args.steps):
            binding.gmc_sample(m, c, integ, K, 2, s * N, out=o)
    elif kind in ("film", "film_rk4"):
        integ, K = ("rk4", 12) if kind == "film_rk4" else ("euler", HEAD_K)
        w = fitted("gmc_film_h512.bin") or inputs.random_film_weights(HEAD_H, 1)
        m = binding.Model(inputs.pack_blob(w), "bf16")
        N = HEAD_N
        c = binding.DeviceCond.from_host(inputs.transmission_conditions(N, 3))
        o = binding.DeviceExit.empty(N)
        for s in range(args.steps):
            binding.gmc_sample(m, c, integ, K, 2, s * N, out=o)
    elif kind == "walk":
        parts = args.profile.split(":")
        tau = float(parts[1]) if len(parts) > 1 else 100.0
        N = (1 << int(parts[2])) if len(parts) > 2 else (1 << 23)
        c = binding.DeviceCond.from_host(inputs.fixed_cell_conditions(N, tau, 1.0, 9))
        o = binding.DeviceExit.empty(N)
        for _ in range(args.steps):
            binding.mc_transmit(c, binding.MODE_CONTINUOUS, 2, 0, out=o)
    elif kind == "lattice_split":
        # the paper's lattice (112^2 cells) with the full method at width 512: births from the
        # internal model, collided crossings from the collided boundary model (RK4 x 12), the
        # uncollided ones streamed through up to 64 cells inside a step
        # (lattice_split:fp8: both models in FP8 e4m3)
        from paper_2512_13965_amd import transport
        mprec = "fp8" if args.profile.split(":")[1:] == ["fp8"] else "bf16"
        col = binding.Model(inputs.pack_blob(fitted("gmc_h512_collided.bin")), mprec)
        src = binding.Model(inputs.pack_blob(fitted("gmc_h512_internal.bin")), mprec)
        w = binding.World(1 << 20, 2, 1 << 14)
        N = 200_000
        walls = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = transport.run_problem(w, inputs.lattice_problem(16), N, 1, binding.SAMPLER_GMC, col, 12,
                                      integrator="rk4", source_model=src, source_K=12, streaming=64)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        w.close()
        col.close()
        src.close()
        print(json.dumps({"lattice_split_s": walls, "precision": mprec, "steps": r["steps"],
                          "transmissions": int(r["transmissions"])}))
    elif kind == "transport":
        from paper_2512_13965_amd import transport
        w = binding.World(1 << 20, 1, 1 << 12)
        for _ in range(args.steps):
            transport.run_problem(w, inputs.checkerboard_problem(32), 200_000, 1, binding.SAMPLER_MC)
        w.close()
        N = 200_000
    else:
        raise SystemExit(f"unknown profile kind {kind}")
    torch.cuda.synchronize()
    print(json.dumps({"profile": args.profile, "launches": args.steps, "batch": N}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--quick", action="store_true", help="only the timed steps")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests in the serving stream")
    ap.add_argument("--detail", default=None, help="file for the full results (JSON)")
    ap.add_argument("--study", default=None, choices=["convergence", "transport", "paper_scale", "thick", "film",
                                                      "serving"],
                    help="run one longer study instead of the benchmark")
    ap.add_argument("--profile", default=None,
                    help="only launch one kernel --steps times: bf16 | fp8 | rk4 | film | film_rk4 (H = 512, 2^20, "
                         "fitted weights) | h128 | h128_rk4 (fitted width 128, 2^20) | fp32 (H = 256, 65,536) | walk:TAU[:LOG2N] | transport | lattice_split[:fp8]")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run plain device copies of 256 MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the sampler shards by particle "
              f"id with no communication between GPUs, and the library runs on a single GPU",
              file=sys.stderr)
        sys.exit(2)
    if args.profile:
        profile_launches(args)
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

    import torch
    from paper_2512_13965_amd import binding, inputs

    w512 = fitted("gmc_h512.bin")
    if w512 is None:
        raise SystemExit("weights/gmc_h512.bin is missing")
    detail_path = args.detail or os.path.join(tempfile.gettempdir(), "gmc_bench_detail.json")
    if args.study:
        fn = {"convergence": lambda: study_convergence(binding, inputs, w512),
              "transport": lambda: study_transport(binding, inputs, w512),
              "paper_scale": lambda: study_paper_scale(binding, inputs, w512),
              "serving": lambda: study_serving(binding, inputs, w512),
              "thick": lambda: study_thick(binding, inputs),
              "film": lambda: study_film(binding, inputs, w512)}[args.study]
        res = {"study": args.study, "result": fn()}
        os.makedirs(os.path.dirname(detail_path), exist_ok=True)
        with open(detail_path, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res))
        return

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    H, K, N = HEAD_H, HEAD_K, HEAD_N
    model = binding.Model(inputs.pack_blob(w512), "bf16")
    cond = binding.DeviceCond.from_host(inputs.transmission_conditions(N, 3), dev)
    out = binding.DeviceExit.empty(N, dev)
    counter = [0]

    def step():
        # a fresh block of particle ids (noise streams) per step
        binding.gmc_transmit(model, cond, K, seed=2, id_base=counter[0] * N, out=out)
        counter[0] += 1

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
    rejected = float((out.face < 0).float().mean().item())
    model.close()
    head = {
        "metric": METRIC, "value": value, "unit": "transmissions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic conditions; weights fitted to this library's analog walk",
        "config": {"workload": "GMC cell-transmission sampler, 2^20 mixed-cell transmissions per launch "
                               "(ln tau~U[ln 0.1, ln 100], c~U[0,1]); velocity MLP 10->512x4->5 SiLU, "
                               "BF16 operands, FP32 accumulation, K=16 Euler steps, fitted weights",
                   "hidden": H, "K": K, "batch": N, "precision": "bf16"},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["bf16"] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK["bf16"], "traffic": measured_traffic(),
                     "kernel": "mlp_ode_kernel<bf16,512,euler>", "avg_launch_ms": float(kms.mean()),
                     "flop_per_launch": fl,
                     "algorithmic_bytes_per_launch": algorithmic_bytes(N, 2 * 796165)},
        "rejected_fraction": rejected,
    }
    log(f"headline: {value:.4e} transmissions/s, kernel {kms.mean():.3f} ms, frac {achieved / PEAK['bf16']:.3f}")
    detail = {"headline": dict(head), "launch_ms": kms.tolist()}
    if args.quick:
        print(json.dumps(head))
        return

    analog = bench_analog(binding, inputs, dev, stream)
    detail["analog"] = analog
    a100 = analog["tps"]["100"]
    head["analog_tps_tau100"] = {"batch_2^23": a100, "batch_2^20": analog["tps_tau100_batch_2^20"]}
    head["gmc_over_analog_tau100"] = value / a100
    head["gmc_over_analog"] = {t: value / analog["tps"][str(int(t))] for t in (1, 10, 100)}
    rows = bench_samplers(binding, inputs, dev, stream, w512)
    detail["samplers"] = rows
    rate = lambda p, integ, k, h=512: next(r["tps"] for r in rows if r["precision"] == p and r["hidden"] == h
                                           and r["integrator"] == integ and r["K"] == k)
    star = {"bf16_h512_euler16": tau_star(value, analog["tps"]),
            "fp8_h512_euler16": tau_star(rate("fp8", "euler", 16), analog["tps"]),
            "bf16_h512_rk4x12": tau_star(rate("bf16", "rk4", 12), analog["tps"])}
    if any(r["hidden"] == 128 for r in rows):
        star["bf16_h128_euler16"] = tau_star(rate("bf16", "euler", 16, 128), analog["tps"])
        star["bf16_h128_rk4x12"] = tau_star(rate("bf16", "rk4", 12, 128), analog["tps"])
    head["tau_star"] = star
    head["fp8_h512_k16"] = {"tps": rate("fp8", "euler", 16),
                            "frac_peak": next(r["frac_peak"] for r in rows if r["precision"] == "fp8"
                                              and r["integrator"] == "euler" and r["K"] == 16)}
    log(f"samplers done; tau* {star}")

    if not args.no_serving:
        sv = bench_serving(binding, inputs, w512, args.serve_requests)
        detail["serving"] = sv
        head["serving"] = {"p50_s": sv["latency_s"]["p50"], "p99_s": sv["latency_s"]["p99"],
                           "requests": sv["requests"], "transmissions_per_s": sv["transmissions_per_s"],
                           "histories_per_request": "1e4-1e7 log-uniform",
                           "load": "70% of measured capacity",
                           "rejected_fraction": sv["rejected_fraction"]}
        log(f"serving p50 {sv['latency_s']['p50']:.3f} s p99 {sv['latency_s']['p99']:.3f} s")

    if not args.no_cpu:
        cb = cpu_baseline(w512, K)
        head["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        detail["cpu_baseline"] = cb
        ca = cpu_baseline_analog()
        detail["cpu_baseline_analog_tau100"] = ca
    dpath = os.path.abspath(detail_path)
    head["detail"] = os.path.relpath(dpath, ROOT) if dpath.startswith(ROOT + os.sep) else dpath
    detail["headline"] = head
    try:
        os.makedirs(os.path.dirname(detail_path), exist_ok=True)
        with open(detail_path, "w") as f:
            json.dump(detail, f, indent=1)
    except OSError as e:
        log(f"could not write {detail_path}: {e}")
    print(json.dumps(head))


if __name__ == "__main__":
    main()
