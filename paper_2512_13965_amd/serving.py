"""Continuous-batching server for transport requests on one GPU.

Each request is an independent transport problem (grid, per-cell materials, source, seed,
number of histories).  Requests that arrive while others are on the device are admitted as soon
as a problem slot and room for their cells (materials + FP64 tallies, a fixed number of bytes
per cell in the world's pool) are free; their source histories are then injected into the
shared particle bank as bank slots free up, so one transport step -- one sampler launch -- works
on particles of every admitted problem at once (the paper's per-particle conditioning makes
mixed-material batches trivial).  A request completes when all its histories have ended; its
tallies are read back and its latency (arrival to tallies on the host) recorded.

Random numbers are keyed by (request seed, history, cell visit), never by bank slot, so a
request's tallies are the same alone and in the mix (up to the order of FP64 atomic additions).
"""
from __future__ import annotations

import heapq
import math
import time
from dataclasses import dataclass, field

import numpy as np

CELL_BYTES = 8 + 8 + 4 + 4 + 9 * 8     # tau, c (FP64), ln tau, c (FP32), 9 FP64 tallies


@dataclass
class Request:
    rid: int
    problem: object            # inputs.Problem
    n_hist: int
    seed: int
    arrival: float = 0.0       # seconds from the start of the run
    # filled by the server
    admitted: float = math.nan
    done: float = math.nan
    tallies: dict | None = None
    transmissions: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def footprint(self) -> int:
        return self.problem.n_cells * CELL_BYTES


@dataclass
class _Active:
    req: Request
    pid: int
    injected: int = 0


@dataclass
class ServeStats:
    requests: list = field(default_factory=list)
    steps: int = 0
    transmissions: int = 0
    wall: float = 0.0

    def latency_percentiles(self, qs=(50, 99)):
        lat = np.array([r.latency for r in self.requests])
        return {f"p{q}": float(np.percentile(lat, q)) for q in qs}

    @property
    def throughput(self) -> float:
        return self.transmissions / self.wall if self.wall > 0 else 0.0


class Server:
    """Admission, injection and stepping over a `binding.World` (or any object with the same
    add_problem / inject / step / alive / tally / remove / capacity interface)."""

    def __init__(self, world, sampler: int, model=None, K: int = 16, cell_budget: int | None = None,
                 chunk: int | None = None, clock=time.perf_counter, sleep=time.sleep,
                 graphs: bool = True):
        self.world = world
        if graphs and hasattr(world, "set_graphs"):
            world.set_graphs(True)      # replay captured steps per batch-size bucket
        self.sampler, self.model, self.K = sampler, model, K
        self.cell_budget = cell_budget            # bytes of cell pool usable by requests
        self.chunk = chunk or max(1, world.capacity // 4)
        self.clock, self.sleep = clock, sleep
        self.active: list[_Active] = []
        self.cells_in_use = 0
        self.alive = 0

    def _try_admit(self, req: Request, now: float) -> bool:
        if self.cell_budget is not None and self.cells_in_use + req.footprint > self.cell_budget:
            return False
        try:
            pid = self.world.add_problem(req.problem, req.seed)
        except Exception as e:          # no free slot or no contiguous room for the cells
            if getattr(e, "code", None) == -2:
                return False
            raise
        req.admitted = now
        self.active.append(_Active(req, pid))
        self.cells_in_use += req.footprint
        return True

    def _inject(self):
        free = self.world.capacity - self.alive
        want = [a for a in self.active if a.injected < a.req.n_hist]
        if not want or free <= 0:
            return
        share = max(1, free // len(want))
        for a in want:
            cnt = min(share, self.chunk, a.req.n_hist - a.injected, self.world.capacity - self.alive)
            if cnt <= 0:
                continue
            self.alive = self.world.inject(a.pid, a.injected, cnt)
            a.injected += cnt

    def _retire(self, now: float, stats: ServeStats):
        keep = []
        for a in self.active:
            if a.injected >= a.req.n_hist and self.world.alive(a.pid) == 0:
                a.req.tallies = self.world.tally(a.pid)
                a.req.done = self.clock() - self._t0
                self.world.remove(a.pid)
                self.cells_in_use -= a.req.footprint
                stats.requests.append(a.req)
            else:
                keep.append(a)
        self.active = keep

    def run(self, requests: list[Request]) -> ServeStats:
        """Serves `requests` (arrival times in seconds from now) to completion."""
        pending = [(r.arrival, r.rid, r) for r in requests]
        heapq.heapify(pending)
        waiting: list[Request] = []          # arrived, not yet admitted (FIFO)
        stats = ServeStats()
        x0 = self.world.transmissions()
        self._t0 = self.clock()
        while pending or waiting or self.active:
            now = self.clock() - self._t0
            while pending and pending[0][0] <= now:
                waiting.append(heapq.heappop(pending)[2])
            while waiting and self._try_admit(waiting[0], now):
                waiting.pop(0)
            if not self.active:
                if waiting:
                    raise RuntimeError(f"request {waiting[0].rid} can never be admitted "
                                       f"({waiting[0].footprint} bytes of cells)")
                if pending:
                    self.sleep(max(0.0, pending[0][0] - (self.clock() - self._t0)))
                continue
            self._inject()
            if self.alive > 0:
                # one launch for every admitted problem's particles
                per = {a.pid: self.world.alive(a.pid) for a in self.active}
                stats.transmissions += self.alive
                for a in self.active:
                    a.req.transmissions += per[a.pid]
                self.alive = self.world.step(self.sampler, self.model, self.K)
                stats.steps += 1
            self._retire(now, stats)
        stats.wall = self.clock() - self._t0
        # cell transmissions, with the first-flight split also those streamed inside steps (the
        # per-request counts are particle-steps)
        stats.transmissions = self.world.transmissions() - x0
        return stats


def poisson_requests(n: int, rate_hz: float, seed: int, make_problem) -> list[Request]:
    """n requests with exponential inter-arrival times of mean 1/rate_hz; make_problem(i)
    returns (problem, n_hist)."""
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate_hz, size=n))
    out = []
    for i in range(n):
        prob, nh = make_problem(i)
        out.append(Request(i, prob, nh, seed=1_000_003 * (i + 1) + seed, arrival=float(t[i])))
    return out
