"""Methods S2 (Section 5.3) and S1 (Section 5.2) on the device, and off-grid
points (needs an MI355X).

With the deterministic method, sdmm_solve_interface builds S_{H,i} of every
Darcy subdomain from each realization's own KL field and solves with it;
sdmm_accumulate_moments then uses those realizations' own responses.  Checked
against the oracle's Method S2 (oracle.methods.Oracle.realization_S2 and
point_S2), element by element:
  * every deterministic S_{H,i} of the batch: 1e-11 (FP64), 1e-10 (mixed);
  * lambda at rtol 1e-12: 1e-9 (FP64), 1e-8 (mixed);
  * the five fields' means and variances: 1e-9 (FP64), 1e-8 (mixed);
  * on collocation points S2 and S3 give the same S blocks, hence the same
    lambda bit for bit (P10 of the oracle pins: S2 = S3 for the same local
    field);
  * off-grid points (seeded N(0,1) draws, Section 2.1: the KL expansion at
    any point of the stochastic space) against the oracle at those points.

With the per-iteration method, sdmm_solve_interface factors each
(subdomain, realization) local problem once and solves it in every CG
iteration; checked against the oracle's Method S1
(oracle.methods.Oracle.realization_S1):
  * lambda and the five fields' means and variances at rtol 1e-12: 1e-9, on
    the two-region layout (all 16 points) and on the small layout with two
    floating Stokes subdomains (FETI), and at off-grid points;
  * the local-solve counter: one solve per Darcy subdomain per CG iteration
    plus one recovery solve per realization (eq. S1-cost);
  * S1, S2 and S3 give the same lambda on collocation points of the
    4x4-Darcy layout to the CG tolerance.
"""
import numpy as np
import pytest

from oracle.darcy import DarcyLocal
from oracle.methods import FIELDS, Oracle
from workloads import problem

from gpu_helpers import rel

pytestmark = pytest.mark.gpu


def _det_ctx(prob, precision):
    import torch  # noqa: F401  (torch's HIP runtime first)
    from paper_1802_06263_amd import sdmm
    ctx = sdmm.Context(0)
    ctx.set_problem(prob)
    ctx.build_flux_basis(precision, method="deterministic")
    return ctx


def _solve(ctx, idx=None, y=None, rtol=1e-12):
    import torch
    M = ctx.sizes()["M"]
    n = len(idx) if idx is not None else y.shape[0]
    g = torch.tensor(np.asarray(idx, dtype=np.int64), device="cuda") if idx is not None else None
    yt = torch.tensor(np.ascontiguousarray(y, dtype=np.float64), device="cuda") if y is not None else None
    lam = torch.zeros((n, M), dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    ctx.solve_interface(g, lam, rtol=rtol, status=st, y=yt)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    return g, yt, lam


def _check_moments(ctx, mom, tol):
    for f in FIELDS:
        mg, vg = ctx.get_moments(f)
        mo, vo = mom[f]
        assert rel(mg, mo) < tol, (f, rel(mg, mo))
        assert np.abs(vg - vo).max() < tol * max(np.abs(vo).max(), 1e-12 * np.abs(mo).max() ** 2), f


@pytest.fixture(scope="module")
def cfg0_s2():
    o = Oracle(problem("cfg0"))
    mom, info = o.run("S2", rtol=1e-12)
    return o, mom, info


@pytest.mark.parametrize("precision,tol_s,tol", [("fp64", 1e-11, 1e-9), ("mixed", 1e-10, 1e-8)])
def test_s2_matches_oracle_cfg0(cfg0_s2, precision, tol_s, tol):
    print("case: Method S2 on the two-region layout", precision, flush=True)
    o, mom, info = cfg0_s2
    ctx = _det_ctx(o.prob, precision)
    n = o.grid.nreal
    g, _, lam = _solve(ctx, idx=np.arange(n))
    # the deterministic bases of realizations 0 and 11
    for q in (0, 11):
        y = o.grid.points[q]
        for i in o.darcy_ids:
            S = o.darcy_local(i, y).basis()
            assert rel(ctx.get_basis(i, q, S.shape[0]), S) < tol_s, (i, q)
    assert rel(lam.cpu().numpy(), np.stack([d["lambda"] for d in info])) < tol
    ctx.reset_moments()
    ctx.accumulate_moments(g, lam)
    _check_moments(ctx, mom, tol)
    c = ctx.counters()
    assert c["basis_solves_darcy"] == n * sum(o.L.sub_dofs[i].size for i in o.darcy_ids)
    ctx.close()


def test_s2_equals_s3_on_collocation_points():
    print("case: S2 and S3 give the same lambda on collocation points", flush=True)
    from gpu_helpers import gpu_ctx, gpu_solve
    prob = problem("cfg1")
    idx = [0, 5, 17, 200, 360]
    c3 = gpu_ctx(prob, "fp64")
    _, lam3, it3, _, _, _ = gpu_solve(c3, idx, rtol=1e-10)
    c3.close()
    c2 = _det_ctx(prob, "fp64")
    _, _, lam2 = _solve(c2, idx=idx, rtol=1e-10)
    c2.close()
    assert np.array_equal(lam2.cpu().numpy(), lam3.cpu().numpy())


@pytest.mark.parametrize("name", ["cfg0", "small"])
def test_offgrid_points_match_oracle(name):
    print("case: off-grid points", name, flush=True)
    import torch
    if name == "small":
        prob = problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})
    else:
        prob = problem(name)
    o = Oracle(prob)
    rng = np.random.default_rng(31)
    nt = o.grid.dim_off[-1]
    Y = rng.standard_normal((5, nt))
    w = rng.uniform(0.5, 1.5, 5)
    w /= w.sum()
    ctx = _det_ctx(prob, "fp64")
    _, yt, lam = _solve(ctx, y=Y)
    acc1, acc2 = {}, {}
    for q in range(Y.shape[0]):
        fields, it, rr, ok = o.point_S2(Y[q], rtol=1e-12)
        assert rel(lam[q].cpu().numpy(), fields["lambda"]) < 1e-9, q
        for f, v in fields.items():
            acc1[f] = acc1.get(f, 0.0) + w[q] * v
            acc2[f] = acc2.get(f, 0.0) + w[q] * v * v
    # one deterministic basis of an off-grid point against the oracle's local problem
    i = o.darcy_ids[0]
    S = o.darcy_local(i, Y[2]).basis()
    assert rel(ctx.get_basis(i, 2, S.shape[0]), S) < 1e-11
    ctx.reset_moments()
    ctx.accumulate_moments(None, lam, torch.tensor(w, device="cuda"), y=yt)
    _check_moments(ctx, {f: (acc1[f], acc2[f] - acc1[f] ** 2) for f in acc1}, 1e-9)
    ctx.close()


def test_offgrid_needs_the_deterministic_method():
    print("case: off-grid points on a stochastic basis are refused", flush=True)
    import torch
    from paper_1802_06263_amd import sdmm
    from gpu_helpers import gpu_ctx
    ctx = gpu_ctx(problem("cfg0"), "fp64")
    y = torch.zeros((2, 4), dtype=torch.float64, device="cuda")
    lam = torch.zeros((2, ctx.sizes()["M"]), dtype=torch.float64, device="cuda")
    with pytest.raises(sdmm.SdmmError) as e:
        ctx.solve_interface(None, lam, y=y)
    assert e.value.code == sdmm.EINVAL
    ctx.close()


def _s1_ctx(prob):
    import torch  # noqa: F401  (torch's HIP runtime first)
    from paper_1802_06263_amd import sdmm
    ctx = sdmm.Context(0)
    ctx.set_problem(prob)
    ctx.build_flux_basis("fp64", method="per_iteration")
    return ctx


@pytest.mark.parametrize("name", ["cfg0", "small"])
def test_s1_matches_oracle(name):
    print("case: Method S1", name, flush=True)
    import torch
    if name == "small":
        prob = problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})
        idx = [0, 17, 4000, 6560]
        w = np.array([0.1, 0.2, 0.3, 0.4])
    else:
        prob = problem(name)
        idx = list(range(16))
        w = None
    o = Oracle(prob)
    mom, info = o.run("S1", indices=idx, weights=w, rtol=1e-12)
    ctx = _s1_ctx(prob)
    before = ctx.counters()["basis_solves_darcy"]
    g, _, lam = _solve(ctx, idx=idx)
    assert rel(lam.cpu().numpy(), np.stack([d["lambda"] for d in info])) < 1e-9
    c = ctx.counters()
    nd = len(o.darcy_ids)
    assert c["basis_solves_darcy"] - before == c["cg_iterations"] * nd
    ctx.reset_moments()
    ctx.accumulate_moments(g, lam, None if w is None else torch.tensor(w, device="cuda"))
    assert ctx.counters()["basis_solves_darcy"] - before == c["cg_iterations"] * nd + len(idx) * nd
    _check_moments(ctx, mom, 1e-9)
    from paper_1802_06263_amd import sdmm
    with pytest.raises(sdmm.SdmmError):
        ctx.get_basis(o.darcy_ids[0], 0, 64)
    ctx.close()


def test_s1_offgrid_points_match_oracle():
    print("case: Method S1 at off-grid points", flush=True)
    import torch
    prob = problem("cfg0")
    o = Oracle(prob)
    rng = np.random.default_rng(37)
    Y = rng.standard_normal((4, o.grid.dim_off[-1]))
    w = np.array([0.4, 0.3, 0.2, 0.1])
    ctx = _s1_ctx(prob)
    _, yt, lam = _solve(ctx, y=Y)
    acc1, acc2 = {}, {}
    for q in range(Y.shape[0]):
        fields, it, rr, ok = o.point_S2(Y[q], rtol=1e-12)
        assert rel(lam[q].cpu().numpy(), fields["lambda"]) < 1e-9, q
        for f, v in fields.items():
            acc1[f] = acc1.get(f, 0.0) + w[q] * v
            acc2[f] = acc2.get(f, 0.0) + w[q] * v * v
    ctx.reset_moments()
    ctx.accumulate_moments(None, lam, torch.tensor(w, device="cuda"), y=yt)
    _check_moments(ctx, {f: (acc1[f], acc2[f] - acc1[f] ** 2) for f in acc1}, 1e-9)
    ctx.close()


def test_s1_s2_s3_agree_on_collocation_points():
    print("case: S1, S2 and S3 on collocation points of the 4x4-Darcy layout", flush=True)
    from gpu_helpers import gpu_ctx, gpu_solve
    prob = problem("cfg1")
    idx = [0, 5, 17, 200, 360]
    c3 = gpu_ctx(prob, "fp64")
    _, lam3, *_ = gpu_solve(c3, idx, rtol=1e-11)
    c3.close()
    c2 = _det_ctx(prob, "fp64")
    _, _, lam2 = _solve(c2, idx=idx, rtol=1e-11)
    c2.close()
    c1 = _s1_ctx(prob)
    _, _, lam1 = _solve(c1, idx=idx, rtol=1e-11)
    c1.close()
    l3 = lam3.cpu().numpy()
    assert rel(lam1.cpu().numpy(), l3) < 1e-8
    assert rel(lam2.cpu().numpy(), l3) < 1e-8
