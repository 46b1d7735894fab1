"""Admission accounting of the request loop, on the CPU with a stand-in solver: requests are
admitted by their arena bound, never more at once than the budget holds (unless nothing else
runs), exactly the charged amount comes back, and every plan is closed."""
import threading
import time

import numpy as np

from paper_1611_03189_amd.serve import Request, RequestLoop


class FakeSolver:
    closed = []
    lock = threading.Lock()

    def __init__(self, r, bound):
        self.r = r
        self.arena_bound = bound

    def close(self):
        with FakeSolver.lock:
            FakeSolver.closed.append(self.r.rid)


class FakeLoop(RequestLoop):
    def __init__(self, bounds, fail_rid=None, **kw):
        super().__init__(solver_factory=lambda r: FakeSolver(r, bounds[r.rid]), **kw)
        self.running = 0
        self.in_use = 0
        self.peak = 0
        self.fail_rid = fail_rid
        self.m = threading.Lock()

    def _execute(self, S, r, stream):
        with self.m:
            self.running += 1
            self.in_use += S.arena_bound
            self.peak = max(self.peak, self.in_use if self.running > 1 else 0)
        time.sleep(0.02)
        with self.m:
            self.running -= 1
            self.in_use -= S.arena_bound
        if r.rid == self.fail_rid:
            raise RuntimeError("planted failure")
        return np.zeros((r.n, 1)), {"iterations": 1, "converged": True, "rel_residual": 0.0}, S.arena_bound


def _reqs(k):
    rp = np.array([0, 1], dtype=np.int64)
    ci = np.array([0], dtype=np.int32)
    return [Request(i, rp, ci, np.ones(1), None, np.ones((1, 1)), arrival=0.001 * i) for i in range(k)]


def test_admission_by_bound_and_exact_release():
    FakeSolver.closed = []
    bounds = {i: b for i, b in enumerate([60, 30, 30, 50, 10, 90, 20, 40, 40, 70])}
    loop = FakeLoop(bounds, slots=4, memory_budget=100)
    out = loop.run(_reqs(10), realtime=False)
    assert [r.rid for r in out.results] == list(range(10))
    assert loop.peak <= 100                       # concurrent requests fit the budget
    assert loop.last_peak_used <= 100 or loop.last_peak_used == max(bounds.values())
    assert loop.last_final_used == 0              # everything charged came back
    assert sorted(FakeSolver.closed) == list(range(10))


def test_request_larger_than_budget_runs_alone():
    FakeSolver.closed = []
    bounds = {0: 500, 1: 10, 2: 10}
    loop = FakeLoop(bounds, slots=3, memory_budget=100)
    out = loop.run(_reqs(3), realtime=True)
    assert len(out.results) == 3 and loop.last_final_used == 0
    big = out.results[0]
    others = out.results[1:]
    assert all(o.t_start >= big.t_done - 1e-6 or o.t_done <= big.t_start + 1e-6 for o in others)


def test_failure_releases_and_closes():
    FakeSolver.closed = []
    bounds = {i: 10 for i in range(6)}
    loop = FakeLoop(bounds, fail_rid=2, slots=2, memory_budget=100)
    try:
        loop.run(_reqs(6), realtime=False)
        raise AssertionError("the planted failure was not raised")
    except RuntimeError as e:
        assert "planted" in str(e)
    assert 2 in FakeSolver.closed
