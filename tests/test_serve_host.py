"""Scheduler logic of the serving loop on the host, with a stub executor
(no GPU): admission by memory footprint, rejection, waiting for memory,
deadlines, cancellation, micro-batch formation and latency accounting."""
import threading
import time

import numpy as np
import pytest

from paper_1709_06999_amd.serve import Request, Server


class StubExecutor:
    """Completes a micro-batch `delay` seconds after launch; result = sum(I)."""

    def __init__(self, per_request_bytes=100, delay=0.01, budget=1000):
        self.per = per_request_bytes
        self.delay = delay
        self.budget = budget
        self.launched = []
        self.max_concurrent_bytes = 0
        self._live = 0
        self._lock = threading.Lock()

    def default_budget(self):
        return self.budget

    def footprint(self, reqs):
        return sum(self.per * (10 if r.dataset == "huge" else 1) for r in reqs)

    def launch(self, reqs, slot):
        with self._lock:
            self._live += self.footprint(reqs)
            self.max_concurrent_bytes = max(self.max_concurrent_bytes, self._live)
        self.launched.append([id(r) for r in reqs])
        return (time.perf_counter() + self.delay, reqs)

    def done(self, h):
        return time.perf_counter() >= h[0]

    def collect(self, h):
        with self._lock:
            self._live -= self.footprint(h[1])
        return [(float(np.sum(r.I)), None) for r in h[1]]


def _req(ds="a", val=1.0, grad=False, **kw):
    return Request(ds, np.full(8, val), 0.0, 1e-7, 64, 1e-7, grad=grad, **kw)


def test_results_and_microbatches():
    ex = StubExecutor(delay=0.02)
    srv = Server(ex, max_batch=4, max_inflight=2).start()
    futs = [srv.submit(_req(val=float(i))) for i in range(10)]
    res = [f.result(timeout=5) for f in futs]
    srv.stop()
    assert [r[0] for r in res] == [8.0 * i for i in range(10)]
    st = srv.stats()
    assert st["completed"] == 10 and st["batches"] < 10      # requests were batched
    assert max(len(b) for b in ex.launched) <= 4
    assert st["p50_ms"] is not None and st["p99_ms"] >= st["p50_ms"]


def test_memory_admission_waits_and_rejects():
    ex = StubExecutor(per_request_bytes=400, delay=0.02, budget=1000)
    srv = Server(ex, max_batch=8, max_inflight=4).start()
    futs = [srv.submit(_req(val=1.0)) for _ in range(6)]
    big = srv.submit(_req(ds="huge"))                          # 4000 bytes > budget
    res = [f.result(timeout=5) for f in futs]
    with pytest.raises(MemoryError):
        big.result(timeout=5)
    srv.stop()
    assert all(r[0] == 8.0 for r in res)
    assert ex.max_concurrent_bytes <= 1000                     # never over budget
    assert max(len(b) for b in ex.launched) <= 2               # at most 2 x 400 fit
    assert srv.stats()["rejected"] == 1


def test_deadline_and_cancellation():
    ex = StubExecutor(per_request_bytes=600, delay=0.05, budget=1000)
    srv = Server(ex, max_batch=1, max_inflight=1).start()
    first = srv.submit(_req(val=2.0))                          # occupies the device
    late = srv.submit(_req(val=3.0, deadline=time.perf_counter() + 0.01))
    cancelled = srv.submit(_req(val=4.0))
    assert cancelled.cancel()
    ok = srv.submit(_req(val=5.0))
    assert first.result(timeout=5)[0] == 16.0
    with pytest.raises(TimeoutError):
        late.result(timeout=5)
    assert ok.result(timeout=5)[0] == 40.0
    srv.stop()
    assert srv.stats()["expired"] == 1
    assert all(id(late) not in b for b in ex.launched)


def test_grad_and_plain_requests_are_not_mixed():
    ex = StubExecutor(delay=0.01)
    srv = Server(ex, max_batch=8, max_inflight=1).start()
    reqs = [_req(val=1.0, grad=(i % 2 == 0)) for i in range(8)]
    futs = [srv.submit(r) for r in reqs]
    [f.result(timeout=5) for f in futs]
    srv.stop()
    byid = {id(r): r for r in reqs}
    for b in ex.launched:
        assert len({byid[i].grad for i in b}) == 1


class MixedStub(StubExecutor):
    mixed_batches = True


def test_mixed_executor_takes_requests_in_arrival_order():
    ex = MixedStub(delay=0.01)
    srv = Server(ex, max_batch=4, max_inflight=1).start()
    reqs = [_req(ds="ab"[i % 2], val=float(i), grad=(i % 3 == 0)) for i in range(12)]
    futs = [srv.submit(r) for r in reqs]
    res = [f.result(timeout=5) for f in futs]
    srv.stop()
    assert [r[0] for r in res] == [8.0 * i for i in range(12)]
    order = [i for b in ex.launched for i in b]
    assert order == [id(r) for r in reqs]                      # FIFO across keys
    assert any(len({reqs[[id(r) for r in reqs].index(i)].key() for i in b}) > 1
               for b in ex.launched)


class PlanningStub(StubExecutor):
    """footprint() raises for requests on dataset 'bad' (as the GPU executor
    does for a request its planner refuses)."""

    def footprint(self, reqs):
        if any(r.dataset == "bad" for r in reqs):
            raise ValueError("planner refused the request")
        return super().footprint(reqs)


def test_request_the_executor_cannot_plan_is_rejected_alone():
    ex = PlanningStub(delay=0.01)
    srv = Server(ex, max_batch=8, max_inflight=2).start()
    futs = [srv.submit(_req(ds="bad" if i == 3 else "a", val=float(i))) for i in range(8)]
    for i, f in enumerate(futs):
        if i == 3:
            with pytest.raises(ValueError, match="planner refused"):
                f.result(timeout=5)
        else:
            assert f.result(timeout=5)[0] == 8.0 * i
    srv.stop()
    st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == 7
