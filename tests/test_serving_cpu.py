"""Host logic of the continuous-batching server, on the CPU with a stand-in world (admission by
footprint, FIFO order, injection into free bank slots, retirement)."""
import numpy as np
import pytest

from paper_2512_13965_amd import inputs, serving


class NoRoom(Exception):
    code = -2


class FakeWorld:
    """Same interface as binding.World; each step ends half (rounded up) of every problem's
    particles; problem slots and a cell pool as on the device."""

    def __init__(self, capacity, slots, cells):
        self.capacity, self.slots, self.cells = capacity, slots, cells
        self.used = {}            # pid -> cells
        self.alive_pp = {}
        self.injected = {}
        self.steps = 0
        self.max_alive = 0
        self.xmit = 0

    def add_problem(self, problem, seed):
        free = [p for p in range(self.slots) if p not in self.used]
        if not free or sum(self.used.values()) + problem.n_cells > self.cells:
            raise NoRoom()
        pid = free[0]
        self.used[pid] = problem.n_cells
        self.alive_pp[pid] = 0
        self.injected[pid] = 0
        return pid

    def inject(self, pid, h0, count):
        assert h0 == self.injected[pid], "histories must be injected in order"
        assert sum(self.alive_pp.values()) + count <= self.capacity
        self.injected[pid] += count
        self.alive_pp[pid] += count
        self.max_alive = max(self.max_alive, sum(self.alive_pp.values()))
        return sum(self.alive_pp.values())

    def transmissions(self):
        return self.xmit

    def step(self, sampler, model, K):
        self.steps += 1
        self.xmit += sum(self.alive_pp.values())
        for p in self.alive_pp:
            self.alive_pp[p] //= 2
        return sum(self.alive_pp.values())

    def alive(self, pid):
        return self.alive_pp[pid]

    def tally(self, pid):
        return {"flux": np.full(self.used[pid], float(self.injected[pid]))}

    def remove(self, pid):
        assert self.alive_pp[pid] == 0
        del self.used[pid]


def _req(i, side, nh, t):
    return serving.Request(i, inputs.checkerboard_problem(side, src=2), nh, seed=i, arrival=t)


def _run(world, reqs, **kw):
    clock = {"t": 0.0}

    def now():
        clock["t"] += 1e-3          # every query advances a simulated clock by 1 ms
        return clock["t"]

    srv = serving.Server(world, sampler=1, clock=now, sleep=lambda s: clock.__setitem__("t", clock["t"] + s), **kw)
    return srv.run(reqs)


def test_all_requests_complete_with_their_histories():
    w = FakeWorld(capacity=1000, slots=3, cells=2000)
    reqs = [_req(i, 8 + 4 * (i % 3), 500 + 300 * i, 0.002 * i) for i in range(8)]
    st = _run(w, reqs)
    assert sorted(r.rid for r in st.requests) == list(range(8))
    for r in st.requests:
        assert r.tallies["flux"][0] == r.n_hist           # every history was injected once
        assert r.admitted >= r.arrival and r.done >= r.admitted
    assert w.max_alive <= 1000 and not w.used


def test_admission_waits_for_cell_budget():
    # each request needs 16 x 16 cells; the budget holds two of them at a time
    w = FakeWorld(capacity=10_000, slots=8, cells=10_000)
    reqs = [_req(i, 16, 2000, 0.0) for i in range(5)]
    budget = 2 * 256 * serving.CELL_BYTES
    st = _run(w, reqs, cell_budget=budget)
    order = sorted(st.requests, key=lambda r: r.admitted)
    assert [r.rid for r in order] == [0, 1, 2, 3, 4]     # FIFO
    for r in order[2:]:                                   # admitted only after an earlier one left
        assert any(o.done <= r.admitted for o in order[:2])


def test_slots_limit_concurrency():
    w = FakeWorld(capacity=10_000, slots=1, cells=100_000)
    reqs = [_req(i, 8, 1000, 0.0) for i in range(3)]
    st = _run(w, reqs)
    spans = sorted((r.admitted, r.done) for r in st.requests)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0


def test_request_that_can_never_fit_is_reported():
    w = FakeWorld(capacity=100, slots=2, cells=100)
    with pytest.raises(RuntimeError, match="never be admitted"):
        _run(w, [_req(0, 16, 10, 0.0)])


def test_poisson_arrivals_and_problem_generator():
    reqs = serving.poisson_requests(200, rate_hz=50.0, seed=3,
                                    make_problem=lambda i: inputs.random_problem(i))
    t = np.array([r.arrival for r in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 50.0) < 4 * (1 / 50.0) / np.sqrt(200)
    sides = np.array([r.problem.nx for r in reqs])
    hist = np.array([r.n_hist for r in reqs])
    assert sides.min() >= 16 and sides.max() <= 128
    assert hist.min() >= 10_000 and hist.max() <= 10_000_000
    taus = np.concatenate([r.problem.tau for r in reqs[:20]])
    assert taus.min() >= 0.1 and taus.max() <= 200.0
    assert len({r.seed for r in reqs}) == 200
