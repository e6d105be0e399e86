"""Serving loop on the device: a mixed stream over three problems; every
answer equals the same request solved alone (bit-exact by design: a
realization's CG does not depend on the batch it rides in)."""
import numpy as np
import pytest

from workloads import problem, serving_stream

pytestmark = pytest.mark.gpu


def test_mixed_stream_answers_match_alone():
    print("case: serving stream cfg1 + small FETI cfg2 + cfg0", flush=True)
    from paper_1802_06263_amd.serve import Engine, Server, footprint_bytes, replay, summarize
    probs = {"cfg0": problem("cfg0"), "cfg1": problem("cfg1"),
             "small": problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})}
    server = Server()
    for name, p in probs.items():
        e = Engine(name, p, max_batch=512)
        server.add(e, footprint_bytes(e.backend.sizes, e.max_batch))
    sizes = {p: server.engines[p].backend.sizes["n_real"] for p in probs}
    stream = serving_stream(seed=4, duration_s=0.5, rate_hz=60.0, max_batch=200, grid_sizes=sizes,
                            problems=tuple(probs))
    reqs = replay(server, stream, speed=1.0)
    out = summarize(reqs, 1.0)
    assert out["answered"] == len(stream) and out["not_converged"] == 0
    assert sum(len(b) for b in (server.engines[p].batches for p in probs)) >= 1
    rng = np.random.default_rng(0)
    for q in rng.choice(len(reqs), min(8, len(reqs)), replace=False):
        r = reqs[q]
        lam, it, st = server.engines[r.problem].backend.solve(r.gidx, 1e-8, False)
        assert np.array_equal(lam, r.lam) and np.array_equal(it, r.iters) and np.array_equal(st, r.status)
    server.close()
