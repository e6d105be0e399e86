"""Scheduling logic of the serving loop on the CPU (a fake CG stream stands in
for the device): iteration-level admission into freed slots, per-request
admission by device bytes, rejection, latency accounting."""
import threading
import time

import numpy as np
import pytest

from paper_1802_06263_amd.serve import Engine, Request, Server, footprint_bytes, replay, request_bytes, summarize


class FakeBackend:
    """A CG stream with `slots` slots: realization g needs g % 4 + 1 check
    groups; lambda[l] = gidx[l] + 0.5 * arange(M).  Records, per run, which
    tickets had realizations in slots."""

    def __init__(self, M=4, slots=1 << 30, delay=0.0, groups_of=None):
        self.M = M
        self.slots = slots
        self.delay = delay
        self.groups_of = groups_of or (lambda g: int(g) % 4 + 1)
        self.queue = []            # (ticket, row, gidx)
        self.inslot = []           # [ticket, row, groups left]
        self.left = {}
        self.req = {}
        self.next = 1
        self.history = []          # per run: set of tickets in slots
        self.gate = threading.Event()
        self.gate.set()

    def request_bytes(self, n):
        return request_bytes(self.M, n)

    def submit(self, gidx):
        t = self.next
        self.next += 1
        self.req[t] = np.asarray(gidx)
        self.left[t] = len(gidx)
        self.queue += [(t, q, g) for q, g in enumerate(gidx)]
        return t

    def run(self, groups):
        self.gate.wait()
        while len(self.inslot) < self.slots and self.queue:
            t, q, g = self.queue.pop(0)
            self.inslot.append([t, q, self.groups_of(g)])
        self.history.append({s[0] for s in self.inslot})
        if self.delay:
            time.sleep(self.delay)
        done = []
        for s in self.inslot:
            s[2] -= 1
            if s[2] == 0:
                self.left[s[0]] -= 1
                if self.left[s[0]] == 0:
                    done.append(s[0])
        self.inslot = [s for s in self.inslot if s[2] > 0]
        return done

    def result(self, ticket, accumulate):
        g = self.req.pop(ticket)
        lam = g[:, None].astype(np.float64) + 0.5 * np.arange(self.M)[None, :]
        return lam, np.full(g.size, 7, np.int32), np.zeros(g.size, np.int32)

    def close(self):
        pass


def test_a_request_joins_the_running_stream_and_overtakes():
    """The second request arrives while the first iterates; it takes free
    slots at the next check and finishes first."""
    be = FakeBackend(slots=10, delay=0.01, groups_of=lambda g: 30 if g < 100 else 1)
    e = Engine("p", None, backend=be)
    e.start()
    long_req = Request(0, "p", np.arange(8), 0.0)
    e.submit(long_req)
    time.sleep(0.05)
    short = Request(1, "p", [100, 101], 0.0)
    e.submit(short)
    assert short.event.wait(5) and long_req.event.wait(5)
    e.close()
    assert short.t_done < long_req.t_done
    assert any(len(h) == 2 for h in be.history)          # both requests shared the slots
    assert np.array_equal(short.lam[:, 0], [100.0, 101.0]) and (short.iters == 7).all()


def test_slots_refill_from_the_queue():
    """More realizations than slots: the stream never holds more than its slots
    and every realization is answered."""
    be = FakeBackend(slots=3)
    e = Engine("p", None, backend=be)
    e.start()
    reqs = [Request(q, "p", np.arange(4) + 10 * q, 0.0) for q in range(3)]
    for r in reqs:
        e.submit(r)
    for r in reqs:
        assert r.event.wait(5)
    e.close()
    for r in reqs:
        assert np.array_equal(r.lam[:, 0], r.gidx.astype(float))
    assert max(len(h) for h in be.history) <= 3


def test_requests_wait_for_device_bytes_then_run():
    """A budget that holds one request's outputs: the second is admitted when
    the first releases its bytes, not rejected."""
    be = FakeBackend(slots=64, delay=0.005)
    one = request_bytes(be.M, 5)
    s = Server(hbm_budget_bytes=one + 10)
    e = Engine("p", None, backend=be)
    s.add(e, 0)
    a = Request(0, "p", np.arange(5), 0.0)
    b = Request(1, "p", np.arange(5) + 20, 0.0)
    e.submit(a)
    e.submit(b)
    assert a.event.wait(5) and b.event.wait(5)
    s.close()
    assert not a.rejected and not b.rejected
    assert b.t_done > a.t_done
    assert all(len(h) <= 1 for h in be.history)           # never both in flight
    assert s.used == 0


def test_admission_rejects_beyond_max_pending():
    be = FakeBackend()
    be.gate.clear()
    s = Server(hbm_budget_bytes=request_bytes(be.M, 6))   # only a fits in flight
    e = Engine("p", None, max_pending=10, backend=be)
    s.add(e, 0)
    a = Request(0, "p", np.arange(6), 0.0)
    b = Request(1, "p", np.arange(6), 0.0)
    c = Request(2, "p", np.arange(4), 0.0)
    assert e.submit(a)
    time.sleep(0.05)            # a is admitted: the queue is empty again
    assert e.submit(b)          # waits for device bytes
    assert not e.submit(Request(3, "p", np.arange(5), 0.0))   # 6 + 5 > 10 waiting
    assert e.submit(c)                                        # 6 + 4 <= 10
    be.gate.set()
    for r in (a, b, c):
        assert r.event.wait(5)
    s.close()


def test_server_admits_engines_by_hbm_footprint():
    s = Server(hbm_budget_bytes=1000)
    e1 = Engine("a", None, backend=FakeBackend())
    s.add(e1, 600)
    with pytest.raises(MemoryError):
        s.add(Engine("b", None, backend=FakeBackend()), 500)
    s.close()
    sizes = {"M": 100, "basis_bytes": 10, "response_bytes": 20}
    assert footprint_bytes(sizes, 2) == 30 + 2 * 8 * (5 * 100 + 16)
    assert request_bytes(100, 3) == 3 * (800 + 8)


def test_replay_and_latency_summary():
    s = Server()
    s.add(Engine("a", None, backend=FakeBackend(delay=0.002)), 0)
    s.add(Engine("b", None, backend=FakeBackend(delay=0.002)), 0)
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


class FakePointBackend:
    """Stands in for the Method S2 backend: run() answers every queued batch
    of points at once; lambda[l] = sum(y_l) + arange(M)."""

    M = 4

    def __init__(self):
        self.pending, self.out, self.next, self.runs = [], {}, 0, []
        self.gate = threading.Event()
        self.gate.set()

    def request_bytes(self, n):
        return request_bytes(self.M, n)

    def submit(self, points):
        assert np.asarray(points).ndim == 2
        self.next += 1
        self.pending.append((self.next, np.asarray(points)))
        return self.next

    def run(self, groups):
        self.gate.wait(5)
        batch, self.pending = self.pending, []
        self.runs.append(len(batch))
        for t, y in batch:
            lam = y.sum(axis=1)[:, None] + np.arange(self.M)[None, :]
            self.out[t] = (lam, np.ones(len(y), np.int32), np.zeros(len(y), np.int32))
        return [t for t, _ in batch]

    def result(self, ticket, accumulate):
        return self.out.pop(ticket)

    def close(self):
        pass


def test_point_requests_are_batched_and_answered():
    """Requests of points y (n x n_term) count n realizations, reach the
    backend as points, and requests queued while a batch runs share the
    next batch."""
    be = FakePointBackend()
    be.gate.clear()
    s = Server(hbm_budget_bytes=1 << 30)
    e = Engine("p", None, backend=be)
    s.add(e, 0)
    rng = np.random.default_rng(3)
    first = Request(0, "p", rng.standard_normal((2, 5)), 0.0)
    assert first.n == 2 and first.points.shape == (2, 5) and first.gidx.size == 0
    e.submit(first)
    time.sleep(0.05)                 # the first batch is running (held at the gate)
    later = [Request(q, "p", rng.standard_normal((q + 1, 5)), 0.0) for q in range(1, 4)]
    for r in later:
        e.submit(r)
    be.gate.set()
    for r in [first] + later:
        assert r.event.wait(5)
        assert np.allclose(r.lam[:, 0], r.points.sum(axis=1))
        assert r.lam.shape == (r.n, be.M)
    s.close()
    assert be.runs[0] == 1 and max(be.runs) == 3   # the three later requests in one batch
    out = summarize([first] + later, 1.0)
    assert out["realizations"] == 2 + 2 + 3 + 4


def test_a_library_error_refuses_the_engines_requests():
    """An error from the backend stops its engine: the requests it holds and
    later ones are refused (their events set), nothing waits forever."""
    class Failing(FakePointBackend):
        def run(self, groups):
            raise RuntimeError("device error")
    be = Failing()
    s = Server(hbm_budget_bytes=1 << 30)
    e = Engine("p", None, backend=be)
    s.add(e, 0)
    a = Request(0, "p", np.zeros((2, 3)), 0.0)
    e.submit(a)
    assert a.event.wait(5) and a.rejected
    b = Request(1, "p", np.zeros((1, 3)), 0.0)
    assert not e.submit(b) and b.rejected
    assert isinstance(e.error, RuntimeError) and s.used == 0
    s.close()
