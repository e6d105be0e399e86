"""Serving loop: batches of collocation realizations against resident flux bases.

A request names a problem and a batch of global collocation indices (the
points of the collocation rule of Section 4); the answer is the mortar
solution lambda of every realization (Section 5.1, CG with S_H applied from
the stochastic basis of Section 5.4), and the realizations are added to the
problem's running moments (Section 2).

Design:
  * one Engine per problem: a library context whose flux basis stays
    resident in HBM, one HIP stream and one worker thread.  Workers spend
    their time inside the C library (ctypes releases the GIL), so requests of
    different problems run concurrently on the device.
  * continuous batching: when its worker is free, an engine takes every
    queued request (oldest first) up to its admitted batch size and solves
    them as one batch.  A realization's result does not depend on the batch
    it rides in (fixed-order reductions in the library), so batching never
    changes answers.
  * admission: engines are admitted only while their resident HBM footprint
    (basis cache, fine responses, CG workspace of one batch) fits the budget;
    a request is rejected when its engine already holds max_pending queued
    realizations.
  * latency is measured from the request's arrival to the end of its batch.

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
    __slots__ = ("rid", "problem", "gidx", "t_arrival", "t_done", "lam", "iters", "status", "rejected", "event")

    def __init__(self, rid, problem, gidx, t_arrival):
        self.rid = rid
        self.problem = problem
        self.gidx = np.asarray(gidx, dtype=np.int64)
        self.t_arrival = t_arrival
        self.t_done = None
        self.lam = None
        self.iters = None
        self.status = None
        self.rejected = False
        self.event = threading.Event()


def footprint_bytes(sizes, batch):
    """Resident device bytes of one engine: basis cache, fine responses and the
    CG state of one batch (r, p, S lambda and lambda itself, M each, and the
    product in the subdomain-local layout, 2 M)."""
    M = sizes["M"]
    per_real = 8 * (6 * M + 64)
    return sizes["basis_bytes"] + sizes["response_bytes"] + batch * per_real


class Engine:
    """One problem on the device: resident basis, a stream and a worker."""

    def __init__(self, name, prob, precision="fp64", max_batch=4096, max_pending=1 << 20, rtol=1e-8,
                 accumulate=True, autotune=True, backend=None):
        self.name = name
        self.rtol = rtol
        self.max_pending = max_pending
        self.accumulate = accumulate
        self.backend = backend if backend is not None else GpuBackend(prob, precision, autotune, max_batch)
        self.max_batch = min(max_batch, self.backend.max_batch)
        self.queue = collections.deque()
        self.pending = 0
        self.cv = threading.Condition()
        self.stop = False
        self.batches = []       # (n_requests, n_realizations, seconds)
        self.thread = threading.Thread(target=self._run, name="engine-" + name, daemon=True)

    def start(self):
        self.thread.start()

    def submit(self, req):
        with self.cv:
            if self.pending + req.gidx.size > self.max_pending:
                req.rejected = True
                req.event.set()
                return False
            self.queue.append(req)
            self.pending += req.gidx.size
            self.cv.notify()
        return True

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify()
        self.thread.join()
        self.backend.close()

    def _take(self):
        batch, n = [], 0
        while self.queue and (not batch or n + self.queue[0].gidx.size <= self.max_batch):
            r = self.queue.popleft()
            batch.append(r)
            n += r.gidx.size
        self.pending -= n
        return batch, n

    def _run(self):
        while True:
            with self.cv:
                while not self.queue and not self.stop:
                    self.cv.wait()
                if self.stop and not self.queue:
                    return
                batch, n = self._take()
            t0 = time.perf_counter()
            gidx = np.concatenate([r.gidx for r in batch])
            lam, iters, status = self.backend.solve(gidx, self.rtol, self.accumulate)
            t1 = time.perf_counter()
            self.batches.append((len(batch), n, t1 - t0))
            off = 0
            for r in batch:
                k = r.gidx.size
                r.lam, r.iters, r.status = lam[off:off + k], iters[off:off + k], status[off:off + k]
                r.t_done = t1
                off += k
                r.event.set()


class GpuBackend:
    """Library context of one problem with its basis built and resident."""

    batch_per_slots = 2   # largest batch, in multiples of the autotuned CG slot count

    def __init__(self, prob, precision, autotune, max_batch):
        import torch
        from . import sdmm
        self.torch = torch
        self.ctx = sdmm.Context(0)
        self.ctx.set_problem(prob)
        # the engines already overlap on the device; lanes would add streams
        # beyond the device's hardware queues
        self.ctx.set_option("cg_lanes", 1)
        self.sizes = self.ctx.sizes()
        self.stream = torch.cuda.Stream()
        self.ctx.build_flux_basis(precision, stream=self.stream)
        self.stream.synchronize()
        self.M = self.sizes["M"]
        self.max_batch = max_batch
        if autotune:
            n = min(self.sizes["n_real"], 8192)
            g = torch.arange(n, dtype=torch.int64, device="cuda")
            # the CG refills its slots from the batch, so a batch may hold more
            # realizations than there are slots without draining between them
            slots = self.ctx.autotune(g, stream=self.stream)
            self.max_batch = min(max_batch, max(256, self.batch_per_slots * slots))
            self.stream.synchronize()

    def solve(self, gidx, rtol, accumulate):
        torch = self.torch
        n = gidx.size
        with torch.cuda.stream(self.stream):
            g = torch.from_numpy(gidx).to("cuda", non_blocking=False)
            lam = torch.empty((n, self.M), dtype=torch.float64, device="cuda")
            it = torch.empty(n, dtype=torch.int32, device="cuda")
            st = torch.empty(n, dtype=torch.int32, device="cuda")
            self.ctx.solve_interface(g, lam, rtol=rtol, iters=it, status=st, stream=self.stream, allow_notconv=True)
            if accumulate:
                self.ctx.accumulate_moments(g, lam, stream=self.stream)
            out = lam.to("cpu", non_blocking=False), it.to("cpu"), st.to("cpu")
        self.stream.synchronize()
        return out[0].numpy(), out[1].numpy(), out[2].numpy()

    def close(self):
        self.stream.synchronize()
        self.ctx.close()


class Server:
    """Engines for several problems plus admission by HBM footprint."""

    def __init__(self, hbm_budget_bytes=200 << 30):
        self.engines = {}
        self.budget = hbm_budget_bytes
        self.used = 0

    def add(self, engine, footprint):
        if self.used + footprint > self.budget:
            raise MemoryError("engine %s needs %d bytes, %d of %d in use" % (engine.name, footprint, self.used,
                                                                           self.budget))
        self.used += footprint
        self.engines[engine.name] = engine
        engine.start()

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
    nreal = int(sum(r.gidx.size for r in done))
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


def build_server(problems, precision, max_batch, budget_gb):
    from workloads import problem
    server = Server(int(budget_gb * (1 << 30)))
    for name in problems:
        e = Engine(name, problem(name), precision=precision, max_batch=max_batch)
        server.add(e, footprint_bytes(e.backend.sizes, e.max_batch))
    return server


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--problems", default="cfg1,cfg2,cfg3")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--duration", type=float, default=10.0, help="seconds of the arrival stream")
    ap.add_argument("--rates", default="200", help="arrival rates (requests/s), comma separated")
    ap.add_argument("--max-batch", type=int, default=8192)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=4)
    args = ap.parse_args(argv)
    from workloads import serving_stream
    problems = tuple(args.problems.split(","))
    server = build_server(problems, args.precision, args.max_batch, args.budget_gb)
    sizes = {p: server.engines[p].backend.sizes["n_real"] for p in problems}

    def log(msg):
        print("serve: " + msg, file=sys.stderr, flush=True)

    for rate in (float(x) for x in args.rates.split(",")):
        stream = serving_stream(seed=args.seed, duration_s=args.duration, rate_hz=rate, grid_sizes=sizes,
                                problems=problems)
        log("rate %.0f/s: %d requests" % (rate, len(stream)))
        t0 = time.perf_counter()
        reqs = replay(server, stream, progress=log)
        out = summarize(reqs, time.perf_counter() - t0)
        out.update({"rate_hz": rate, "offered_realizations_per_s": sum(g.size for _, _, g in stream) / args.duration,
                    "precision": args.precision, "duration_s": args.duration,
                    "max_batch": {p: server.engines[p].max_batch for p in problems}})
        print(json.dumps(out), flush=True)
    server.close()


if __name__ == "__main__":
    main()
