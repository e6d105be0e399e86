"""Scheduling logic of the serving loop on the CPU (a fake backend stands in
for the device): continuous batching, admission, latency accounting."""
import threading
import time

import numpy as np
import pytest

from paper_1802_06263_amd.serve import Engine, Request, Server, footprint_bytes, replay, summarize


class FakeBackend:
    """lambda[l] = gidx[l] + 0.5 * arange(M); records every batch."""

    def __init__(self, M=4, delay=0.0, max_batch=1 << 30):
        self.M = M
        self.delay = delay
        self.max_batch = max_batch
        self.calls = []
        self.gate = threading.Event()
        self.gate.set()

    def solve(self, gidx, rtol, accumulate):
        self.gate.wait()
        self.calls.append(gidx.copy())
        if self.delay:
            time.sleep(self.delay)
        lam = gidx[:, None].astype(np.float64) + 0.5 * np.arange(self.M)[None, :]
        return lam, np.full(gidx.size, 7, np.int32), np.zeros(gidx.size, np.int32)

    def close(self):
        pass


def test_queued_requests_are_batched_up_to_the_limit():
    be = FakeBackend()
    be.gate.clear()
    e = Engine("p", None, max_batch=10, backend=be)
    e.start()
    first = Request(0, "p", [1], 0.0)
    e.submit(first)
    time.sleep(0.05)           # the worker holds the first request at the gate
    reqs = [Request(q + 1, "p", np.arange(4) + 10 * q, 0.0) for q in range(4)]
    for r in reqs:
        e.submit(r)
    be.gate.set()
    for r in [first] + reqs:
        assert r.event.wait(5)
    e.close()
    sizes = [c.size for c in be.calls]
    assert sizes[0] == 1 and all(s <= 10 for s in sizes) and sum(sizes) == 17
    assert sizes[1:] == [8, 8]          # two queued requests per batch of at most 10
    for r in reqs:
        assert np.array_equal(r.lam[:, 0], r.gidx.astype(float))
        assert (r.iters == 7).all() and (r.status == 0).all()


def test_oversized_single_request_still_runs():
    be = FakeBackend()
    e = Engine("p", None, max_batch=3, backend=be)
    e.start()
    r = Request(0, "p", np.arange(8), 0.0)
    e.submit(r)
    assert r.event.wait(5)
    e.close()
    assert [c.size for c in be.calls] == [8]


def test_admission_rejects_beyond_max_pending():
    be = FakeBackend()
    be.gate.clear()
    e = Engine("p", None, max_batch=100, max_pending=10, backend=be)
    e.start()
    a = Request(0, "p", np.arange(6), 0.0)
    b = Request(1, "p", np.arange(6), 0.0)
    c = Request(2, "p", np.arange(4), 0.0)
    assert e.submit(a)
    time.sleep(0.05)            # a is being solved: the queue is empty again
    assert e.submit(b)
    assert not e.submit(Request(3, "p", np.arange(5), 0.0))   # 6 + 5 > 10
    assert e.submit(c)                                        # 6 + 4 <= 10
    be.gate.set()
    for r in (a, b, c):
        assert r.event.wait(5)
    e.close()


def test_server_admits_engines_by_hbm_footprint():
    s = Server(hbm_budget_bytes=1000)
    e1 = Engine("a", None, backend=FakeBackend())
    s.add(e1, 600)
    with pytest.raises(MemoryError):
        s.add(Engine("b", None, backend=FakeBackend()), 500)
    s.close()
    sizes = {"M": 100, "basis_bytes": 10, "response_bytes": 20}
    assert footprint_bytes(sizes, 2) == 30 + 2 * 8 * (6 * 100 + 64)


def test_replay_and_latency_summary():
    s = Server()
    s.add(Engine("a", None, backend=FakeBackend(delay=0.01)), 0)
    s.add(Engine("b", None, backend=FakeBackend(delay=0.01)), 0)
    stream = [(0.001 * q, "a" if q % 2 else "b", np.arange(q % 5 + 1)) for q in range(40)]
    t0 = time.perf_counter()
    reqs = replay(s, stream)
    out = summarize(reqs, time.perf_counter() - t0)
    s.close()
    assert out["answered"] == 40 and out["rejected"] == 0
    assert out["realizations"] == sum(q % 5 + 1 for q in range(40))
    assert 0 < out["latency_p50_ms"] <= out["latency_p99_ms"]
    assert set(out["per_problem"]) == {"a", "b"}
    assert all(r.t_done >= r.t_arrival for r in reqs)
