"""Serving loop: requests of collocation realizations against resident flux bases.

A request names a problem and a batch of global collocation indices (the
points of the collocation rule of Section 4); the answer is the mortar
solution lambda of every realization (Section 5.1, CG with S_H applied from
the stochastic basis of Section 5.4), and the realizations are added to the
problem's running moments (Section 2).  An engine built with --offgrid takes
points y of the stochastic space instead (any draw, e.g. iid N(0, 1)): it
solves each batch of queued points with the deterministic basis of every
realization (Method S2, Section 5.3), so its batching is per batch of
requests, not per CG iteration, and it answers lambda without adding to the
moments (off-grid draws carry no collocation weights).

Design:
  * one Engine per problem: a library context whose flux basis stays
    resident in HBM, one HIP stream, one CG stream of the library
    (sdmm_stream_*) and one worker thread.  Workers spend their time inside
    the C library (ctypes releases the GIL), so requests of different
    problems run concurrently on the device.
  * continuous batching at the level of CG iterations: the CG stream keeps a
    fixed number of slots (the autotuned count); at every convergence check
    (64 iterations) finished realizations leave their slots and realizations
    of any queued request take the freed ones.  A request that arrives while
    others iterate starts at the next check, not after a whole batch.  A
    realization's result does not depend on what shares the slots with it
    (fixed-order reductions in the library), so batching never changes
    answers.
  * admission by HBM footprint, per request: a request enters its engine's
    CG stream only while the device bytes it holds (its lambda and status
    outputs) fit in the budget left after every engine's resident footprint
    (basis cache, fine responses, CG stream workspace); otherwise it waits
    and is admitted as completed requests release their bytes.  A request is
    rejected when its engine already holds max_pending waiting realizations.
  * latency is measured from the request's arrival to its completion.

Run ``python -m paper_1802_06263_amd.serve --help``.
"""
import argparse
import collections
import json
import sys
import threading
import time

import numpy as np


class Request:
    __slots__ = ("rid", "problem", "gidx", "points", "n", "t_arrival", "t_done", "lam", "iters", "status",
                 "rejected", "event", "footprint")

    def __init__(self, rid, problem, gidx, t_arrival):
        """gidx: global collocation indices (1-D), or points y of the
        stochastic space (n x n_term floats) for an off-grid engine."""
        self.rid = rid
        self.problem = problem
        g = np.asarray(gidx)
        if g.ndim == 2:
            self.points = np.ascontiguousarray(g, dtype=np.float64)
            self.gidx = np.zeros(0, dtype=np.int64)
            self.n = g.shape[0]
        else:
            self.points = None
            self.gidx = g.astype(np.int64)
            self.n = self.gidx.size
        self.t_arrival = t_arrival
        self.t_done = None
        self.lam = None
        self.iters = None
        self.status = None
        self.rejected = False
        self.event = threading.Event()
        self.footprint = 0


def footprint_bytes(sizes, slots):
    """Resident device bytes of one engine: basis cache, fine responses and
    the workspace of a CG stream with `slots` slots (r, p, lambda, M each,
    the product in the subdomain-local layout, about 2 M, and per-slot
    scalars)."""
    M = sizes["M"]
    per_slot = 8 * (5 * M + 16)
    return sizes["basis_bytes"] + sizes["response_bytes"] + slots * per_slot


def request_bytes(M, n):
    """Device bytes a request of n realizations holds while in flight: its
    lambda (n x M) and iteration-count and status outputs."""
    return n * (8 * M + 8)


class Engine:
    """One problem on the device: resident basis, a CG stream and a worker."""

    def __init__(self, name, prob, precision="fp64", max_pending=1 << 20, rtol=1e-8, accumulate=True,
                 autotune=True, slots=None, backend=None):
        self.name = name
        self.max_pending = max_pending
        self.accumulate = accumulate
        self.backend = backend if backend is not None else GpuBackend(prob, precision, autotune, slots, rtol)
        self.queue = collections.deque()
        self.pending = 0          # realizations waiting for admission
        self.inflight = {}        # ticket -> request (worker thread only)
        self.cv = threading.Condition()
        self.stop = False
        self.server = None
        self.runs = []            # per CG check group: (requests in flight, realizations in flight, seconds)
        self.error = None         # the library error that stopped the engine, if any
        self.thread = threading.Thread(target=self._run, name="engine-" + name, daemon=True)

    def start(self):
        self.thread.start()

    def submit(self, req):
        with self.cv:
            if self.error is not None or self.pending + req.n > self.max_pending:
                req.rejected = True
                req.event.set()
                return False
            self.queue.append(req)
            self.pending += req.n
            self.cv.notify()
        return True

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify()
        self.thread.join()
        self.backend.close()

    def _admit(self):
        """Queued requests into the CG stream while their bytes fit (oldest first)."""
        while self.queue:
            r = self.queue[0]
            fp = self.backend.request_bytes(r.n)
            if self.server is not None and not self.server.reserve(fp):
                break
            self.queue.popleft()
            self.pending -= r.n
            r.footprint = fp
            self.inflight[self.backend.submit(r.gidx if r.points is None else r.points)] = r

    def _run(self):
        while True:
            with self.cv:
                while not self.queue and not self.inflight and not self.stop:
                    self.cv.wait()
                if self.stop and not self.queue and not self.inflight:
                    return
                self._admit()
                if not self.inflight:
                    self.cv.wait(0.001)   # every queued request waits for device memory
                    continue
            nreq = len(self.inflight)
            nreal = sum(r.n for r in self.inflight.values())
            t0 = time.perf_counter()
            try:
                done = self.backend.run(1)
                t1 = time.perf_counter()
                self.runs.append((nreq, nreal, t1 - t0))
                for t in done:
                    r = self.inflight.pop(t)
                    r.lam, r.iters, r.status = self.backend.result(t, self.accumulate)
                    r.t_done = time.perf_counter()
                    if self.server is not None:
                        self.server.release(r.footprint)
                    r.event.set()
            except Exception as exc:   # a library error ends this engine: every request it holds is refused
                self.error = exc
                with self.cv:
                    held = list(self.inflight.values()) + list(self.queue)
                    self.inflight.clear()
                    self.queue.clear()
                    self.pending = 0
                    self.stop = True
                for r in held:
                    if r.footprint and self.server is not None:
                        self.server.release(r.footprint)
                    r.rejected = True
                    r.event.set()
                return


class GpuBackend:
    """Library context of one problem with its basis resident and one CG stream."""

    def __init__(self, prob, precision, autotune, slots, rtol):
        import torch
        from . import sdmm
        self.torch = torch
        self.ctx = sdmm.Context(0)
        self.ctx.set_problem(prob)
        self.sizes = self.ctx.sizes()
        self.stream = torch.cuda.Stream()
        self.ctx.build_flux_basis(precision, stream=self.stream)
        self.stream.synchronize()
        self.M = self.sizes["M"]
        if slots is None:
            if autotune:
                # requests repeat points, so the sample is 8192 realizations even
                # when the grid has fewer points (the slots then fill with repeats)
                g = torch.arange(8192, dtype=torch.int64, device="cuda") % self.sizes["n_real"]
                slots = self.ctx.autotune(g, stream=self.stream)
                self.stream.synchronize()
            else:
                slots = 1024
        self.slots = slots
        self.sid = self.ctx.stream_open(slots, rtol=rtol, stream=self.stream)
        self.out = {}

    def request_bytes(self, n):
        return request_bytes(self.M, n)

    def submit(self, gidx):
        torch = self.torch
        n = gidx.size
        lam = torch.empty((n, self.M), dtype=torch.float64, device="cuda")
        it = torch.empty(n, dtype=torch.int32, device="cuda")
        st = torch.empty(n, dtype=torch.int32, device="cuda")
        t = self.ctx.stream_submit(self.sid, gidx, lam, iters=it, status=st)
        self.out[t] = (gidx, lam, it, st)
        return t

    def run(self, groups):
        done, _ = self.ctx.stream_run(self.sid, groups)
        return done

    def result(self, ticket, accumulate):
        torch = self.torch
        gidx, lam, it, st = self.out.pop(ticket)
        with torch.cuda.stream(self.stream):
            if accumulate:
                g = torch.from_numpy(gidx).to("cuda", non_blocking=False)
                self.ctx.accumulate_moments(g, lam, stream=self.stream)
            out = lam.to("cpu"), it.to("cpu"), st.to("cpu")
        self.stream.synchronize()
        return out[0].numpy(), out[1].numpy(), out[2].numpy()

    def solve_alone(self, gidx, rtol):
        """The same realizations through sdmm_solve_interface (for checks)."""
        torch = self.torch
        n = gidx.size
        with torch.cuda.stream(self.stream):
            g = torch.from_numpy(np.asarray(gidx, dtype=np.int64)).to("cuda")
            lam = torch.empty((n, self.M), dtype=torch.float64, device="cuda")
            it = torch.empty(n, dtype=torch.int32, device="cuda")
            st = torch.empty(n, dtype=torch.int32, device="cuda")
            self.ctx.solve_interface(g, lam, rtol=rtol, iters=it, status=st, stream=self.stream, allow_notconv=True)
            out = lam.to("cpu"), it.to("cpu"), st.to("cpu")
        self.stream.synchronize()
        return out[0].numpy(), out[1].numpy(), out[2].numpy()

    def close(self):
        self.stream.synchronize()
        self.ctx.stream_close(self.sid)
        self.ctx.close()


class PointBackend:
    """Library context of one problem under Method S2: every batch of queued
    points y is solved at once, each realization with its own Darcy basis
    built from its KL field (sdmm_solve_interface with y).  It answers
    lambda only: the moments of off-grid draws need weights that a stream
    does not fix (1/N for N iid draws), so the caller accumulates them."""

    def __init__(self, prob, precision, rtol):
        import torch
        from . import sdmm
        self.torch = torch
        self.ctx = sdmm.Context(0)
        self.ctx.set_problem(prob)
        self.sizes = self.ctx.sizes()
        self.stream = torch.cuda.Stream()
        self.ctx.build_flux_basis(precision, method="deterministic", stream=self.stream)
        self.stream.synchronize()
        self.M = self.sizes["M"]
        self.rtol = rtol
        self.slots = 0
        # device bytes per realization of a batch: lambda and outputs, and its
        # own Darcy bases and fine responses (the stochastic basis per unit
        # times the Darcy subdomains)
        self.per_real = request_bytes(self.M, 1) + (self.sizes["basis_bytes"] + self.sizes["response_bytes"]) * \
            self.sizes["n_darcy"] // max(1, self.sizes["n_units"])
        self.pending = []
        self.out = {}
        self.next = 0

    def request_bytes(self, n):
        return n * self.per_real

    def submit(self, points):
        t = self.next
        self.next += 1
        self.pending.append((t, np.asarray(points, dtype=np.float64)))
        return t

    def run(self, groups):
        if not self.pending:
            return []
        torch = self.torch
        batch, self.pending = self.pending, []
        Y = np.concatenate([y for _, y in batch])
        n = Y.shape[0]
        with torch.cuda.stream(self.stream):
            y = torch.from_numpy(Y).to("cuda")
            lam = torch.empty((n, self.M), dtype=torch.float64, device="cuda")
            it = torch.empty(n, dtype=torch.int32, device="cuda")
            st = torch.empty(n, dtype=torch.int32, device="cuda")
            self.ctx.solve_interface(None, lam, rtol=self.rtol, iters=it, status=st, stream=self.stream, y=y,
                                     allow_notconv=True)
            out = lam.to("cpu").numpy(), it.to("cpu").numpy(), st.to("cpu").numpy()
        self.stream.synchronize()
        q = 0
        for t, yb in batch:
            k = yb.shape[0]
            self.out[t] = tuple(a[q:q + k] for a in out)
            q += k
        return [t for t, _ in batch]

    def result(self, ticket, accumulate):
        return self.out.pop(ticket)

    def solve_alone(self, points, rtol):
        """The same points as a batch of their own (for checks)."""
        torch = self.torch
        Y = np.ascontiguousarray(points, dtype=np.float64)
        n = Y.shape[0]
        with torch.cuda.stream(self.stream):
            y = torch.from_numpy(Y).to("cuda")
            lam = torch.empty((n, self.M), dtype=torch.float64, device="cuda")
            it = torch.empty(n, dtype=torch.int32, device="cuda")
            st = torch.empty(n, dtype=torch.int32, device="cuda")
            self.ctx.solve_interface(None, lam, rtol=rtol, iters=it, status=st, stream=self.stream, y=y,
                                     allow_notconv=True)
            out = lam.to("cpu").numpy(), it.to("cpu").numpy(), st.to("cpu").numpy()
        self.stream.synchronize()
        return out

    def close(self):
        self.stream.synchronize()
        self.ctx.close()


class Server:
    """Engines for several problems plus admission by HBM footprint: every
    engine's resident bytes when it is added, every request's bytes while it
    is in flight."""

    def __init__(self, hbm_budget_bytes=200 << 30):
        self.engines = {}
        self.budget = hbm_budget_bytes
        self.used = 0
        self.lock = threading.Lock()

    def add(self, engine, footprint):
        with self.lock:
            if self.used + footprint > self.budget:
                raise MemoryError("engine %s needs %d bytes, %d of %d in use" % (engine.name, footprint, self.used,
                                                                               self.budget))
            self.used += footprint
        self.engines[engine.name] = engine
        engine.server = self
        engine.start()

    def reserve(self, nbytes):
        with self.lock:
            if self.used + nbytes > self.budget:
                return False
            self.used += nbytes
            return True

    def release(self, nbytes):
        with self.lock:
            self.used -= nbytes
        for e in self.engines.values():
            with e.cv:
                e.cv.notify()

    def submit(self, req):
        return self.engines[req.problem].submit(req)

    def close(self):
        for e in self.engines.values():
            e.close()


def replay(server, stream, speed=1.0, progress=None):
    """Submit (t, problem, gidx) requests at their arrival times (divided by
    speed) and wait for all answers.  Returns the requests."""
    reqs = [Request(q, p, g, t / speed) for q, (t, p, g) in enumerate(stream)]
    t0 = time.perf_counter()
    for r in reqs:
        dt = r.t_arrival - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        r.t_arrival += t0
        server.submit(r)
    last = time.perf_counter()
    for q, r in enumerate(reqs):
        r.event.wait()
        if progress is not None and time.perf_counter() - last > 10.0:
            progress("%d of %d requests answered" % (q + 1, len(reqs)))
            last = time.perf_counter()
    return reqs


def summarize(reqs, wall_s):
    done = [r for r in reqs if not r.rejected]
    lat = np.array([r.t_done - r.t_arrival for r in done]) if done else np.zeros(1)
    nreal = int(sum(r.n for r in done))
    out = {"requests": len(reqs), "answered": len(done), "rejected": len(reqs) - len(done),
           "realizations": nreal, "wall_s": wall_s, "realizations_per_s": nreal / wall_s,
           "latency_p50_ms": float(np.percentile(lat, 50) * 1e3), "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
           "not_converged": int(sum(int((r.status != 0).sum()) for r in done))}
    per = collections.defaultdict(list)
    for r in done:
        per[r.problem].append(r.t_done - r.t_arrival)
    out["per_problem"] = {p: {"requests": len(v), "p50_ms": float(np.percentile(v, 50) * 1e3),
                              "p99_ms": float(np.percentile(v, 99) * 1e3)} for p, v in sorted(per.items())}
    return out


def build_server(problems, precision, budget_gb, offgrid=False, rtol=1e-8):
    from workloads import problem
    server = Server(int(budget_gb * (1 << 30)))
    for name in problems:
        if offgrid:
            e = Engine(name, problem(name), backend=PointBackend(problem(name), precision, rtol))
        else:
            e = Engine(name, problem(name), precision=precision, rtol=rtol)
        server.add(e, footprint_bytes(e.backend.sizes, e.backend.slots))
    return server


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--problems", default="cfg1,cfg2,cfg3")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--duration", type=float, default=10.0, help="seconds of the arrival stream")
    ap.add_argument("--rates", default="200", help="arrival rates (requests/s), comma separated")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--offgrid", action="store_true",
                    help="requests of iid N(0, 1) points of the stochastic space (Method S2 engines)")
    args = ap.parse_args(argv)
    from workloads import serving_stream
    problems = tuple(args.problems.split(","))
    server = build_server(problems, args.precision, args.budget_gb, offgrid=args.offgrid)
    sizes = {p: server.engines[p].backend.sizes["n_real"] for p in problems}
    nterm = {p: server.engines[p].backend.sizes["n_term"] for p in problems}

    def log(msg):
        print("serve: " + msg, file=sys.stderr, flush=True)

    for rate in (float(x) for x in args.rates.split(",")):
        stream = serving_stream(seed=args.seed, duration_s=args.duration, rate_hz=rate, grid_sizes=sizes,
                                problems=problems)
        if args.offgrid:
            # the same arrivals and request sizes, each realization an iid
            # N(0, 1) point of the problem's stochastic space
            rng = np.random.default_rng(args.seed + 1)
            stream = [(t, p, rng.standard_normal((g.size, nterm[p]))) for t, p, g in stream]
        log("rate %.0f/s: %d requests" % (rate, len(stream)))
        t0 = time.perf_counter()
        reqs = replay(server, stream, progress=log)
        out = summarize(reqs, time.perf_counter() - t0)
        out.update({"rate_hz": rate, "offered_realizations_per_s": sum(len(g) for _, _, g in stream) / args.duration,
                    "precision": args.precision, "duration_s": args.duration, "offgrid": args.offgrid,
                    "cg_slots": {p: server.engines[p].backend.slots for p in problems},
                    "requests_in_flight_per_check": {
                        p: float(np.mean([x[0] for x in server.engines[p].runs] or [0])) for p in problems}})
        for e in server.engines.values():
            e.runs.clear()
        print(json.dumps(out), flush=True)
    server.close()


if __name__ == "__main__":
    main()
