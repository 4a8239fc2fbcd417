"""Server scheduling logic on the CPU, with a fake backend behind the same
interface the GPU backend implements: admission by memory footprint, slot
limits, arrival order, rejection, failure isolation, overflow re-issue and
latency bookkeeping."""
import time

import numpy as np

from paper_1410_4803_amd.serve import Request, Server, poisson_requests


class FakeBackend:
    def __init__(self, service_s=0.002, fail_on=(), overflow_once=()):
        self.service_s = service_s
        self.fail_on = set(fail_on)
        self.overflow_once = set(overflow_once)
        self.started = []
        self.concurrent = 0
        self.max_concurrent = 0

    def footprint(self, req):
        return 1000 * len(req.sample_idx) + (10 if req.ld_capacity else 0)

    def start(self, req, slot):
        if req.rid in self.fail_on:
            raise RuntimeError("injected backend failure")
        self.started.append(req.rid)
        self.concurrent += 1
        self.max_concurrent = max(self.max_concurrent, self.concurrent)
        return {"t": time.perf_counter() + self.service_s, "slot": slot}

    def poll(self, h):
        return time.perf_counter() >= h["t"]

    def finish(self, req, h):
        self.concurrent -= 1
        if req.rid in self.overflow_once and not req.ld_capacity:
            req.ld_capacity = 99
            return False
        req.device_ms = self.service_s * 1e3
        req.result = int(req.sample_idx.sum()) + req.v_range[0]
        return True


def _reqs(sizes, arrival=0.0):
    return [Request(k, "ibs" if k % 3 else "ld", 0, np.arange(s, dtype=np.int32), (k, k + 100),
                    arrival=arrival) for k, s in enumerate(sizes)]


def test_admission_respects_budget_and_slots():
    be = FakeBackend(service_s=0.003)
    srv = Server(be, n_slots=3, memory_budget=250_000)
    reqs = _reqs([100] * 10)                   # 100 kB each: at most 2 fit the budget
    stats = srv.run(reqs)
    assert stats["completed"] == 10 and stats["rejected"] == 0
    assert srv.peak_used <= 250_000
    assert be.max_concurrent == 2
    assert be.started == list(range(10))       # arrival order
    assert stats["memory_holds"] >= 1          # the budget, not the slots, held requests
    assert all(r.result == int(np.arange(100).sum()) + r.rid for r in srv.finished)
    for key in ("p50_ms", "p99_ms", "throughput_rps", "queue_wait_p99_ms"):
        assert key in stats


def test_slots_bound_concurrency():
    be = FakeBackend(service_s=0.003)
    srv = Server(be, n_slots=4, memory_budget=10 ** 12)
    srv.run(_reqs([10] * 20))
    assert be.max_concurrent == 4 and srv.max_running == 4


def test_rejects_oversized_and_survives_failures():
    be = FakeBackend(fail_on={2})
    srv = Server(be, n_slots=2, memory_budget=50_000)
    reqs = _reqs([10, 20, 30, 100, 5])          # rid 3 needs 100 kB > budget
    stats = srv.run(reqs)
    done = sorted(r.rid for r in srv.finished)
    assert done == [0, 1, 4]
    errs = {r.rid: r.error for r in srv.rejected}
    assert "budget" in errs[3] and "injected" in errs[2]
    assert stats["completed"] == 3 and stats["rejected"] == 2


def test_overflow_is_reissued():
    be = FakeBackend(overflow_once={1, 4})
    srv = Server(be, n_slots=2, memory_budget=10 ** 9)
    srv.run(_reqs([10] * 6))
    assert sorted(r.rid for r in srv.finished) == list(range(6))
    assert be.started.count(1) == 2 and be.started.count(4) == 2
    assert all(r.ld_capacity == 99 for r in srv.finished if r.rid in (1, 4))


def test_poisson_workload_shape():
    shapes = [(1000, 10000), (50000, 200000)]
    reqs = poisson_requests(shapes, rate=200, seconds=5, seed=1)
    assert 800 < len(reqs) < 1200
    assert all(np.all(np.diff(r.sample_idx) > 0) for r in reqs)   # distinct, sorted
    for r in reqs:
        n, V = shapes[r.cohort]
        assert 100 <= len(r.sample_idx) <= min(5000, n)
        assert 0 <= r.v_range[0] < r.v_range[1] <= V
        assert 1000 <= r.v_range[1] - r.v_range[0] <= min(20000, V)
    frac_ibs = np.mean([r.kind == "ibs" for r in reqs])
    assert 0.65 < frac_ibs < 0.75
    arr = np.array([r.arrival for r in reqs])
    assert (np.diff(arr) > 0).all() and arr[-1] <= 5


class GrowingOverflowBackend(FakeBackend):
    """An LD request whose overflow size makes its footprint exceed the budget."""

    def footprint(self, req):
        return 1000 if not req.ld_capacity else 10 ** 7


def test_overflow_beyond_budget_is_rejected():
    be = GrowingOverflowBackend(overflow_once={1})
    srv = Server(be, n_slots=2, memory_budget=100_000)
    stats = srv.run(_reqs([10] * 4))            # run() must return
    assert sorted(r.rid for r in srv.finished) == [0, 2, 3]
    errs = {r.rid: r.error for r in srv.rejected}
    assert list(errs) == [1] and "budget" in errs[1]
    assert stats["completed"] == 3 and stats["rejected"] == 1 and srv.idle()
