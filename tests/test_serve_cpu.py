"""CPU tests of the serving scheduler with a mock executor (no GPU):
admission by footprint, deferral and release, rejection, cancellation,
continuous batching at step boundaries."""
import numpy as np
import pytest

from paper_1609_07757_amd.serve import Request, Server, ci_dim, davidson_bytes


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt):
        self.t += dt


class MockExecutor:
    """Each request needs `iters = norb // 10` steps; a step costs 1 ms."""

    def __init__(self, clock, fp=None):
        self.clock = clock
        self.left = {}
        self.req = {}
        self.running_max = 0
        self.log = []
        self.fp = fp or (lambda r: r.norb * 1000)

    def footprint(self, r):
        return self.fp(r)

    def start(self, r):
        tok = r.rid
        self.left[tok] = max(1, r.norb // 10)
        self.req[tok] = r
        self.log.append(("start", r.rid, self.clock.t))
        return tok

    def step(self):
        self.clock.advance(1e-3)
        self.running_max = max(self.running_max, len(self.left))
        for t in self.left:
            self.left[t] -= 1
        return len(self.left)

    def poll(self, tok):
        done = self.left[tok] <= 0
        return done, np.array([-float(self.req[tok].norb)]), {"iterations": 1}

    def finish(self, tok):
        del self.left[tok]
        self.log.append(("finish", tok, self.clock.t))


def _reqs(n, gap=0.002, norbs=None):
    norbs = norbs or [20 + (7 * i) % 50 for i in range(n)]
    return [Request(i, i * gap, norbs[i], 2, 2, 2, 1e-12, 1) for i in range(n)]


def test_all_served_and_energies_routed():
    clk = FakeClock()
    ex = MockExecutor(clk)
    srv = Server(ex, hbm_budget=10**9, clock=clk)
    done = srv.run(_reqs(30))
    assert len(done) == 30 and all(r.status == "done" for r in done)
    for r in done:
        assert r.energies[0] == -r.norb
        assert r.latency > 0
    rep = srv.report()
    assert rep["served"] == 30 and rep["p99_s"] >= rep["p50_s"]


def test_budget_never_exceeded_and_requests_defer():
    clk = FakeClock()
    ex = MockExecutor(clk)
    budget = 100_000          # about two requests of norb ~50
    srv = Server(ex, hbm_budget=budget, clock=clk)
    reqs = _reqs(20, gap=0.0)
    done = srv.run(reqs)
    assert all(r.status == "done" for r in done)
    assert srv.peak_used <= budget
    assert ex.running_max <= 3
    # arrival order is kept: starts are in rid order (FIFO admission)
    starts = [rid for kind, rid, _ in ex.log if kind == "start"]
    assert starts == sorted(starts)


def test_continuous_batching_joins_mid_flight():
    clk = FakeClock()
    ex = MockExecutor(clk)
    srv = Server(ex, hbm_budget=10**9, clock=clk)
    # a long request, then short ones arriving while it runs
    reqs = [Request(0, 0.0, 200, 2, 2, 3, 1e-12, 1)] + [Request(i, 0.003 * i, 20, 2, 2, 2, 1e-12, 1)
                                                         for i in range(1, 6)]
    done = {r.rid: r for r in srv.run(reqs)}
    assert ex.running_max >= 2
    # short requests finished before the long one although they came later
    assert all(done[i].finished < done[0].finished for i in range(1, 6))


def test_oversized_request_rejected_not_blocking():
    clk = FakeClock()
    ex = MockExecutor(clk)
    srv = Server(ex, hbm_budget=50_000, clock=clk)
    reqs = [Request(0, 0.0, 100, 2, 2, 2, 0.0, 1), Request(1, 0.0, 20, 2, 2, 2, 0.0, 1)]
    done = {r.rid: r for r in srv.run(reqs)}
    assert done[0].status == "rejected"
    assert done[1].status == "done"


def test_cancel_queued_and_running():
    clk = FakeClock()
    ex = MockExecutor(clk)
    srv = Server(ex, hbm_budget=30_000, clock=clk)
    srv._t0 = 0.0
    srv.queue.extend(_reqs(3, norbs=[20, 20, 20]))
    srv._admit()
    assert len(srv.running) == 1 and len(srv.queue) == 2
    assert srv.cancel(2)           # queued
    assert srv.cancel(0)           # running: memory released
    assert srv.used == 0
    srv._admit()
    assert [r.rid for r, _ in srv.running.values()] == [1]


def test_slot_limit():
    clk = FakeClock()
    ex = MockExecutor(clk)
    srv = Server(ex, hbm_budget=10**12, max_slots=4, clock=clk)
    srv.run(_reqs(12, gap=0.0))
    assert ex.running_max <= 4


def test_footprint_model():
    assert ci_dim(106, 2, 2, 2) == 54393
    b1 = davidson_bytes(1000, 1)
    b4 = davidson_bytes(1000, 4)
    assert 0 < b1 < b4
    assert davidson_bytes(10**6, 1) >= 8 * 10**6 * 32


def test_size_class_time_share():
    """The executor's class choice gives the fast class its share of step
    time while both classes have solves, and the busy class otherwise."""
    from paper_1609_07757_amd.serve import pick_class
    assert pick_class([1, 0], [0.0, 0.0], 0.75) == 0
    assert pick_class([0, 3], [5.0, 0.0], 0.75) == 1
    # simulated steps: fast steps cost 1, slow steps cost 10
    active, t, n = [4, 2], [0.0, 0.0], [0, 0]
    for _ in range(4000):
        c = pick_class(active, t, 0.75)
        t[c] += 1.0 if c == 0 else 10.0
        n[c] += 1
    assert abs(t[0] / (t[0] + t[1]) - 0.75) < 0.01
    assert n[0] > 25 * n[1]


class OomExecutor(MockExecutor):
    """Builds fail with MemoryError while `busy` other solves run above
    `limit` (an estimate that was too low); running solves are charged a
    held size different from the admission estimate."""

    def __init__(self, clock, limit):
        super().__init__(clock, fp=lambda r: 1000)
        self.limit = limit
        self.fails = 0

    def start(self, r):
        if len(self.left) >= self.limit:
            self.fails += 1
            raise MemoryError("device out of memory")
        return super().start(r)

    def charge(self, tok):
        return 700 + tok


def test_oom_build_requeues_and_charges_held_bytes():
    clk = FakeClock()
    ex = OomExecutor(clk, limit=2)
    srv = Server(ex, hbm_budget=10_000, max_slots=8, clock=clk)
    reqs = _reqs(6, gap=0.0, norbs=[30] * 6)
    done = srv.run(reqs)
    assert sorted(r.rid for r in done if r.status == "done") == list(range(6))
    assert ex.fails >= 1 and srv.report()["oom_requeued"] == ex.fails
    assert ex.running_max <= 2
    # requests start in arrival order despite the failed builds
    starts = [rid for kind, rid, _ in ex.log if kind == "start"]
    assert starts == sorted(starts)
    assert srv.used == 0


def test_oom_with_nothing_running_rejects():
    clk = FakeClock()
    ex = OomExecutor(clk, limit=0)
    srv = Server(ex, hbm_budget=10_000, max_slots=8, clock=clk)
    done = srv.run(_reqs(2, gap=0.0, norbs=[30, 30]))
    assert all(r.status == "rejected" for r in done) and len(done) == 2
