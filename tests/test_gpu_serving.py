"""Serving loop on the device: a mixed stream over three problems.  Requests
join the running CG stream of their problem at convergence checks, so
several requests share its slots; every answer equals the same request
solved alone through sdmm_solve_interface (bit-exact by design: a
realization's CG does not depend on what shares the slots with it)."""
import numpy as np
import pytest

from workloads import problem, serving_stream

pytestmark = pytest.mark.gpu


def test_mixed_stream_answers_match_alone():
    print("case: serving stream cfg1 + small FETI cfg2 + cfg0 through CG streams", flush=True)
    from paper_1802_06263_amd.serve import Engine, Server, footprint_bytes, replay, summarize
    probs = {"cfg0": problem("cfg0"), "cfg1": problem("cfg1"),
             "small": problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})}
    server = Server()
    for name, p in probs.items():
        e = Engine(name, p, slots=256)
        server.add(e, footprint_bytes(e.backend.sizes, e.backend.slots))
    sizes = {p: server.engines[p].backend.sizes["n_real"] for p in probs}
    stream = serving_stream(seed=4, duration_s=0.5, rate_hz=60.0, max_batch=200, grid_sizes=sizes,
                            problems=tuple(probs))
    reqs = replay(server, stream, speed=1.0)
    out = summarize(reqs, 1.0)
    assert out["answered"] == len(stream) and out["not_converged"] == 0
    # some check group carried realizations of two or more requests
    shared = max(max((x[0] for x in server.engines[p].runs), default=0) for p in probs)
    print("  most requests sharing one CG stream at a check: %d" % shared, flush=True)
    assert shared >= 2
    for r in reqs:
        lam, it, st = server.engines[r.problem].backend.solve_alone(r.gidx, 1e-8)
        assert np.array_equal(lam, r.lam) and np.array_equal(it, r.iters) and np.array_equal(st, r.status)
    server.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_layouts_in_the_mix_match_alone(precision):
    """The two large serving layouts (4x2 Stokes over 8x4 Darcy 64x64, and the
    uneven P2 layout) served together: every answer equals the same request
    solved alone, in both precisions."""
    print("case: serving stream on the full cfg2 + cfg3 layouts,", precision, flush=True)
    from paper_1802_06263_amd.serve import Engine, Server, footprint_bytes, replay, summarize
    names = ("cfg2", "cfg3")
    server = Server()
    for name in names:
        e = Engine(name, problem(name), precision=precision, slots=1024)
        server.add(e, footprint_bytes(e.backend.sizes, e.backend.slots))
    sizes = {p: server.engines[p].backend.sizes["n_real"] for p in names}
    stream = serving_stream(seed=5, duration_s=0.25, rate_hz=48.0, max_batch=96, grid_sizes=sizes, problems=names)
    reqs = replay(server, stream, speed=1.0)
    out = summarize(reqs, 1.0)
    assert out["answered"] == len(stream) and out["not_converged"] == 0
    shared = max(max((x[0] for x in server.engines[p].runs), default=0) for p in names)
    print("  %d requests; most sharing one CG stream at a check: %d" % (len(stream), shared), flush=True)
    assert shared >= 2
    for r in reqs:
        lam, it, st = server.engines[r.problem].backend.solve_alone(r.gidx, 1e-8)
        assert np.array_equal(lam, r.lam) and np.array_equal(it, r.iters) and np.array_equal(st, r.status)
    server.close()


def test_offgrid_point_requests_match_alone():
    """Requests of iid N(0, 1) points through a Method S2 engine: queued
    requests share a batch, and every answer is bit for bit the answer of
    its points solved as a batch of their own."""
    print("case: serving off-grid points through a Method S2 engine (two-region layout)", flush=True)
    from paper_1802_06263_amd.serve import Engine, PointBackend, Request, Server
    prob = problem("cfg0")
    be = PointBackend(prob, "fp64", 1e-10)
    s = Server(1 << 34)
    e = Engine("cfg0", prob, backend=be)
    s.add(e, 0)
    rng = np.random.default_rng(5)
    nt = be.sizes["n_term"]
    reqs = [Request(q, "cfg0", rng.standard_normal((q + 2, nt)), 0.0) for q in range(4)]
    for r in reqs:
        s.submit(r)
    for r in reqs:
        assert r.event.wait(120)
    runs = list(e.runs)
    alone = [be.solve_alone(r.points, 1e-10) for r in reqs]
    s.close()
    assert max(x[0] for x in runs) >= 2, runs
    for r, (lam, it, st) in zip(reqs, alone):
        assert (r.status == 0).all() and (st == 0).all()
        assert np.array_equal(r.lam, lam), r.rid
