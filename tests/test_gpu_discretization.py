"""Discretization variants of Section 6 on the device (needs an MI355X): the
triangular Taylor-Hood pair and the exactly integrated RT0 mass.

Triangular Taylor-Hood (P2-P1, two triangles per rectangle on the Q2-Q1 node
grid) against the oracle's StokesLocal with the same element:
  * every Stokes S_{H,i} (FP64 band LDL^T, one refinement step): 1e-11
    relative to max|S|, the bar of the Q2-Q1 blocks;
  * lambda and the five fields' means and variances at rtol 1e-12: 1e-9,
    on the two-region layout and on the small layout with two floating
    Stokes subdomains (FETI);
  * at full size (4x2 Stokes subdomains of 64x64 elements), the S blocks of
    one Stokes subdomain on the outer boundary and of one floating one;
  * Methods S2 and S1 with the P2-P1 element on the two-region layout:
    lambda and the five fields at rtol 1e-12 against the oracle's S2 / S1,
    1e-9.
"""
import numpy as np
import pytest

from oracle.geometry import Layout
from oracle.methods import FIELDS, Oracle
from oracle.stokes import StokesLocal
from workloads import problem

from gpu_helpers import gpu_ctx, gpu_solve, rel

pytestmark = pytest.mark.gpu


def _with(prob, **disc):
    prob = dict(prob)
    prob["discretization"] = dict(disc)
    return prob


def _small_feti():
    return problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})


def _check_moments(ctx, mom, tol):
    for f in FIELDS:
        mg, vg = ctx.get_moments(f)
        mo, vo = mom[f]
        assert rel(mg, mo) < tol, (f, rel(mg, mo))
        assert np.abs(vg - vo).max() < tol * max(np.abs(vo).max(), 1e-12 * np.abs(mo).max() ** 2), f


@pytest.mark.parametrize("name", ["cfg0", "small"])
def test_p2p1_matches_oracle(name):
    print("case: P2-P1 Stokes element,", name, flush=True)
    import torch
    prob = _with(_small_feti() if name == "small" else problem("cfg0"), stokes="p2p1")
    o = Oracle(prob)
    o.stochastic_basis()
    ctx = gpu_ctx(prob, "fp64")
    for i in o.stokes_ids:
        S = o.s3_table[(i, 0)]
        assert rel(ctx.get_basis(i, 0, S.shape[0]), S) < 1e-11, i
    if name == "small":
        assert ctx.sizes()["n_kernel"] == 4
        idx, w = [0, 17, 4000, 6560], np.array([0.1, 0.2, 0.3, 0.4])
    else:
        idx, w = list(range(o.grid.nreal)), None
    g, lam, it, rr, st, rc = gpu_solve(ctx, idx, rtol=1e-12)
    assert (st == 0).all()
    mom, info = o.run("S3", indices=idx, weights=w, rtol=1e-12)
    assert rel(lam.cpu().numpy(), np.stack([d["lambda"] for d in info])) < 1e-9
    ctx.accumulate_moments(g, lam, None if w is None else torch.tensor(w, device="cuda"))
    _check_moments(ctx, mom, 1e-9)
    ctx.close()


def test_p2p1_full_size_stokes_blocks():
    print("case: P2-P1 Stokes blocks on the 4x2 layout of 64x64 elements", flush=True)
    prob = _with(problem("cfg2"), stokes="p2p1")
    L = Layout(prob)
    ctx = gpu_ctx(prob, "fp64")
    floating = [i for i in range(L.n_stokes) if L.is_floating(i)]
    assert floating
    for i in (0, floating[0]):
        S = StokesLocal(L, i).basis()
        assert rel(ctx.get_basis(i, 0, S.shape[0]), S) < 1e-11, i
    ctx.close()



@pytest.mark.parametrize("method", ["S2", "S1"])
def test_p2p1_methods_s1_s2_match_oracle(method):
    print("case: P2-P1 Stokes element under Method", method, "on the two-region layout", flush=True)
    import torch
    from paper_1802_06263_amd import sdmm
    prob = _with(problem("cfg0"), stokes="p2p1")
    o = Oracle(prob)
    idx = [1, 6, 11]
    w = np.array([0.5, 0.3, 0.2])
    mom, info = o.run(method, indices=idx, weights=w, rtol=1e-12)
    ctx = sdmm.Context(0)
    ctx.set_problem(prob)
    ctx.build_flux_basis("fp64", method="deterministic" if method == "S2" else "per_iteration")
    M = ctx.sizes()["M"]
    gi = torch.tensor(idx, dtype=torch.int64, device="cuda")
    lam = torch.zeros((len(idx), M), dtype=torch.float64, device="cuda")
    st = torch.zeros(len(idx), dtype=torch.int32, device="cuda")
    ctx.solve_interface(gi, lam, rtol=1e-12, status=st)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    assert rel(lam.cpu().numpy(), np.stack([d["lambda"] for d in info])) < 1e-9
    ctx.reset_moments()
    ctx.accumulate_moments(gi, lam, torch.tensor(w, device="cuda"))
    _check_moments(ctx, mom, 1e-9)
    ctx.close()

# ---- exactly integrated RT0 mass (hybridized face-pressure system) ----------
#   * every Darcy S_{H,i}^{(k)} (FP64 band Cholesky of the face-pressure
#     system, no refinement): 1e-11 relative to max|S|;
#   * lambda and the five fields at rtol 1e-12: 1e-9, with Methods S3 and S2
#     (the two-region and the small FETI layouts), and lambda at off-grid
#     points under Method S2;
#   * on the 4x2 Stokes over 8x4 Darcy layout with 48x48 Darcy meshes
#     (the largest that fits the factor's LDS window: band 2 min(nx, ny) + 1),
#     sampled units of three Darcy subdomains;
#   * at full size (64x64 Darcy subdomains, band 129: the tiled band LDL^T),
#     sampled units, and on the uneven layout one unit of every mesh shape
#     (window and tiled units in one build); the CG converges at full size;
#   * the mixed precision path and Method S1 refuse the exact mass (EINVAL);
#   * Method S2 at full size (tiled units alone, and tiled with window units
#     in one batch): lambda on collocation points agrees with Method S3's,
#     and every sampled unit with the oracle's basis;
#   * both variants together (P2-P1 Stokes, exact-mass Darcy) on the
#     two-region layout: every S block, lambda and the moments.


@pytest.mark.parametrize("name", ["cfg0", "small"])
def test_exact_rt0_matches_oracle(name):
    print("case: exact RT0 mass,", name, flush=True)
    import torch
    prob = _with(_small_feti() if name == "small" else problem("cfg0"), darcy="exact")
    o = Oracle(prob)
    o.stochastic_basis()
    ctx = gpu_ctx(prob, "fp64")
    for (i, k), S in o.s3_table.items():
        if i in o.darcy_ids and (name == "cfg0" or k in (0, 4, 8)):
            assert rel(ctx.get_basis(i, k, S.shape[0]), S) < 1e-11, (i, k, rel(ctx.get_basis(i, k, S.shape[0]), S))
    if name == "small":
        idx, w = [0, 17, 4000, 6560], np.array([0.1, 0.2, 0.3, 0.4])
    else:
        idx, w = list(range(o.grid.nreal)), None
    g, lam, it, rr, st, rc = gpu_solve(ctx, idx, rtol=1e-12)
    assert (st == 0).all()
    mom, info = o.run("S3", indices=idx, weights=w, rtol=1e-12)
    assert rel(lam.cpu().numpy(), np.stack([d["lambda"] for d in info])) < 1e-9
    ctx.accumulate_moments(g, lam, None if w is None else torch.tensor(w, device="cuda"))
    _check_moments(ctx, mom, 1e-9)
    ctx.close()


def test_both_variants_together_match_oracle():
    print("case: P2-P1 Stokes with the exact RT0 mass on the two-region layout", flush=True)
    prob = _with(problem("cfg0"), stokes="p2p1", darcy="exact")
    o = Oracle(prob)
    o.stochastic_basis()
    ctx = gpu_ctx(prob, "fp64")
    for (i, k), S in o.s3_table.items():
        assert rel(ctx.get_basis(i, k, S.shape[0]), S) < 1e-11, (i, k)
    idx = list(range(o.grid.nreal))
    g, lam, it, rr, st, rc = gpu_solve(ctx, idx, rtol=1e-12)
    mom, info = o.run("S3", indices=idx, rtol=1e-12)
    assert rel(lam.cpu().numpy(), np.stack([d["lambda"] for d in info])) < 1e-9
    ctx.accumulate_moments(g, lam)
    _check_moments(ctx, mom, 1e-9)
    ctx.close()


@pytest.mark.parametrize("name", ["cfg0", "small"])
def test_exact_rt0_method_s2_matches_oracle(name):
    print("case: exact RT0 mass, Method S2,", name, flush=True)
    import torch
    from paper_1802_06263_amd import sdmm
    prob = _with(_small_feti() if name == "small" else problem("cfg0"), darcy="exact")
    o = Oracle(prob)
    idx = [0, 17, 4000, 6560] if name == "small" else [1, 6, 11]
    w = np.array([0.1, 0.2, 0.3, 0.4]) if name == "small" else np.array([0.5, 0.3, 0.2])
    mom, info = o.run("S2", indices=idx, weights=w, rtol=1e-12)
    ctx = sdmm.Context(0)
    ctx.set_problem(prob)
    ctx.build_flux_basis("fp64", method="deterministic")
    M = ctx.sizes()["M"]
    gi = torch.tensor(idx, dtype=torch.int64, device="cuda")
    lam = torch.zeros((len(idx), M), dtype=torch.float64, device="cuda")
    st = torch.zeros(len(idx), dtype=torch.int32, device="cuda")
    ctx.solve_interface(gi, lam, rtol=1e-12, status=st)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    assert rel(lam.cpu().numpy(), np.stack([d["lambda"] for d in info])) < 1e-9
    ctx.reset_moments()
    ctx.accumulate_moments(gi, lam, torch.tensor(w, device="cuda"))
    _check_moments(ctx, mom, 1e-9)
    ctx.close()



def test_exact_rt0_offgrid_points_match_oracle():
    print("case: exact RT0 mass, Method S2 at off-grid points of the two-region layout", flush=True)
    import torch
    from paper_1802_06263_amd import sdmm
    prob = _with(problem("cfg0"), darcy="exact")
    o = Oracle(prob)
    rng = np.random.default_rng(41)
    Y = rng.standard_normal((3, o.grid.dim_off[-1]))
    ctx = sdmm.Context(0)
    ctx.set_problem(prob)
    ctx.build_flux_basis("fp64", method="deterministic")
    M = ctx.sizes()["M"]
    y = torch.tensor(Y, dtype=torch.float64, device="cuda")
    lam = torch.zeros((Y.shape[0], M), dtype=torch.float64, device="cuda")
    st = torch.zeros(Y.shape[0], dtype=torch.int32, device="cuda")
    ctx.solve_interface(None, lam, rtol=1e-12, status=st, y=y)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for q in range(Y.shape[0]):
        fields, it, rr, ok = o.point_S2(Y[q], rtol=1e-12)
        assert rel(lam[q].cpu().numpy(), fields["lambda"]) < 1e-9, q
    ctx.close()

def test_exact_rt0_sampled_units_48x48():
    print("case: exact RT0 mass, sampled units of the 8x4 Darcy layout at 48x48", flush=True)
    from oracle.collocation import Grid
    from oracle.darcy import DarcyLocalExact
    from oracle.kl import cell_centres, region_field
    prob = _with(problem("cfg2", darcy_mesh=(48, 48)), darcy="exact")
    L = Layout(prob)
    grid = Grid(prob["regions"], prob["rule"])
    ctx = gpu_ctx(prob, "fp64")
    darcy = [i for i in range(L.nsub) if L.subs[i]["type"] == "darcy"]
    rng = np.random.default_rng(13)
    for i in (darcy[0], darcy[len(darcy) // 2], darcy[-1]):
        sub = L.subs[i]
        reg = L.regions[sub["region"]]
        k = int(rng.integers(grid.nlocal[sub["region"]]))
        y = grid.local_points(sub["region"])[k]
        K = np.exp(float(reg["mean_logk"]) + np.asarray(y) @ region_field(reg, cell_centres(sub)))
        S = DarcyLocalExact(L, i, K).basis()
        assert rel(ctx.get_basis(i, k, S.shape[0]), S) < 1e-11, (i, k)
    ctx.close()


def test_exact_rt0_refuses_mixed_and_s1():
    print("case: exact RT0 mass refuses mixed precision and Method S1", flush=True)
    import torch  # noqa: F401
    from paper_1802_06263_amd import sdmm
    ctx = sdmm.Context(0)
    ctx.set_problem(_with(problem("cfg0"), darcy="exact"))
    for prec, meth in (("mixed", "stochastic"), ("fp64", "per_iteration")):
        with pytest.raises(sdmm.SdmmError) as e:
            ctx.build_flux_basis(prec, method=meth)
        assert e.value.code == sdmm.EINVAL
    ctx.close()


def _exact_unit_basis(L, grid, i, k):
    from oracle.darcy import DarcyLocalExact
    from oracle.kl import cell_centres, region_field
    sub = L.subs[i]
    reg = L.regions[sub["region"]]
    y = grid.local_points(sub["region"])[k]
    K = np.exp(float(reg["mean_logk"]) + np.asarray(y) @ region_field(reg, cell_centres(sub)))
    return DarcyLocalExact(L, i, K).basis()


@pytest.mark.parametrize("name", ["cfg2", "cfg3"])
def test_exact_rt0_full_size_units(name):
    print("case: exact RT0 mass at full size,", name, flush=True)
    import torch
    from oracle.collocation import Grid
    prob = _with(problem(name), darcy="exact")
    L = Layout(prob)
    grid = Grid(prob["regions"], prob["rule"])
    ctx = gpu_ctx(prob, "fp64")
    darcy = [i for i in range(L.nsub) if L.subs[i]["type"] == "darcy"]
    rng = np.random.default_rng(17)
    if name == "cfg3":
        seen = {}
        for i in darcy:
            seen.setdefault(tuple(L.subs[i]["n"]), i)
        subs = list(seen.values())
    else:
        subs = [darcy[0], darcy[len(darcy) // 2], darcy[-1]]
    for i in subs:
        k = int(rng.integers(grid.nlocal[L.subs[i]["region"]]))
        S = _exact_unit_basis(L, grid, i, k)
        assert rel(ctx.get_basis(i, k, S.shape[0]), S) < 1e-11, (i, k, L.subs[i]["n"])
    idx = [int(v) for v in rng.integers(0, grid.nreal, 64)]
    g, lam, it, rr, st, rc = gpu_solve(ctx, idx, rtol=1e-8)
    assert (st == 0).all() and (rr <= 1e-8).all()
    # Method S2 builds each realization's own units through the same
    # tiled path: lambda on collocation points agrees with Method S3's,
    # and the unit of batch position 0 with the oracle's basis
    few = idx[:8]
    gi = torch.tensor(few, dtype=torch.int64, device="cuda")
    lam3 = torch.zeros((len(few), lam.shape[1]), dtype=torch.float64, device="cuda")
    ctx.solve_interface(gi, lam3, rtol=1e-12)
    ctx.build_flux_basis("fp64", method="deterministic")
    lam2 = torch.zeros_like(lam3)
    st2 = torch.zeros(len(few), dtype=torch.int32, device="cuda")
    ctx.solve_interface(gi, lam2, rtol=1e-12, status=st2)
    torch.cuda.synchronize()
    assert (st2.cpu().numpy() == 0).all()
    assert rel(lam2.cpu().numpy(), lam3.cpu().numpy()) < 1e-10
    from oracle.darcy import DarcyLocalExact
    from oracle.kl import cell_centres, region_field
    for i in subs:
        sub = L.subs[i]
        r = sub["region"]
        yr = np.asarray(grid.points[few[0]])[grid.dim_off[r]:grid.dim_off[r + 1]]
        K = np.exp(float(L.regions[r]["mean_logk"]) + yr @ region_field(L.regions[r], cell_centres(sub)))
        S = DarcyLocalExact(L, i, K).basis()
        assert rel(ctx.get_basis(i, 0, S.shape[0]), S) < 1e-11, (i, sub["n"])
    ctx.close()
