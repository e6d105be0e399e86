"""Full-size parity of the HIP path (needs an MI355X).

cfg1 is small enough for the oracle to run whole: every realization through
Method S3 at rtol 1e-13, compared field by field with the GPU moments.  On
cfg2 and cfg3 the oracle computes sampled flux bases one by one (one unit
per Darcy mesh shape on cfg3, i.e. every shape class of the launch), and the
CG and moment results are checked through properties that hold at any size:

  * the true FETI-projected residual P (g - S lambda) of every sampled
    realization, recomputed on the host in FP64 from the library's own
    S blocks (pinned by the sampled bases), g and G, is at most 2e-8 ||P g||
    (the CG stops on its recursive residual, which differs from the true one
    by rounding), and G^T lambda = 0;
  * the mean and variance of lambda equal the weighted sums of the returned
    realizations (Section 2 with the collocation weights of Section 4).

Tolerances for S and the moments are those of test_gpu_parity.
"""
import numpy as np
import pytest

from oracle import interface as itf
from oracle.collocation import Grid
from oracle.darcy import DarcyLocal
from oracle.geometry import Layout
from oracle.kl import cell_centres, region_field
from oracle.methods import FIELDS, Oracle
from workloads import problem

from gpu_helpers import gpu_ctx, gpu_solve, rel

pytestmark = pytest.mark.gpu


def oracle_unit_basis(L, grid, i, k):
    """S_{H,i}^{(k)} of one Darcy unit by the oracle (Section 5.4)."""
    sub = L.subs[i]
    reg = L.regions[sub["region"]]
    phi = region_field(reg, cell_centres(sub))
    y = grid.local_points(sub["region"])[k]
    K = np.exp(float(reg["mean_logk"]) + np.asarray(y) @ phi)
    return DarcyLocal(L, i, K).basis()


def sampled_units(L, grid, name, rng):
    darcy = [i for i in range(L.nsub) if L.subs[i]["type"] == "darcy"]
    if name == "cfg3":
        # one unit per Darcy mesh shape: every shape class of the launch
        seen = {}
        for i in darcy:
            seen.setdefault(tuple(L.subs[i]["n"]), i)
        subs = list(seen.values())
    else:
        subs = [darcy[0], darcy[len(darcy) // 2], darcy[-1]]
    return [(i, int(rng.integers(grid.nlocal[L.subs[i]["region"]]))) for i in subs]


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("mixed", 1e-10)])
def test_sampled_basis_parity_full_size(name, precision, tol):
    print("case: sampled basis", name, precision, flush=True)
    prob = problem(name)
    L = Layout(prob)
    grid = Grid(prob["regions"], prob["rule"])
    ctx = gpu_ctx(prob, precision)
    if precision == "mixed":
        assert ctx.counters()["max_refine_residual"] <= 1e-11
    rng = np.random.default_rng(11)
    for i, k in sampled_units(L, grid, name, rng):
        S = oracle_unit_basis(L, grid, i, k)
        Sg = ctx.get_basis(i, k, S.shape[0])
        assert rel(Sg, S) < tol, (name, i, k, rel(Sg, S))
    ctx.close()


@pytest.fixture(scope="module")
def cfg1_oracle_loop():
    o = Oracle(problem("cfg1"))
    # rtol 1e-13 on both sides: at 1e-12 the two CGs stop at points whose
    # difference, amplified by the Stokes pressure recovery, reaches 1e-9
    mom, info = o.run("S3", rtol=1e-13)
    return o, mom, info


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-8)])
def test_cfg1_all_realizations_match_oracle(cfg1_oracle_loop, precision, tol):
    print("case: cfg1 full collocation loop vs oracle", precision, flush=True)
    o, mom, info = cfg1_oracle_loop
    ctx = gpu_ctx(o.prob, precision)
    g_h, _ = ctx.interface_data()
    assert rel(g_h, o.g_stokes) < 1e-11
    n = o.grid.nreal
    g, lam, it, rr, st, rc = gpu_solve(ctx, np.arange(n), rtol=1e-13)
    assert (st == 0).all()
    lam_o = np.stack([d["lambda"] for d in info])
    assert rel(lam.cpu().numpy(), lam_o) < tol
    ctx.accumulate_moments(g, lam)
    for f in FIELDS:
        mg, vg = ctx.get_moments(f)
        mo, vo = mom[f]
        assert rel(mg, mo) < tol, f
        assert np.abs(vg - vo).max() < tol * max(np.abs(vo).max(), 1e-12 * np.abs(mo).max() ** 2), f
    ctx.close()


def _assembled_S(ctx, L, g2l, l):
    S_loc = []
    for i in range(L.nsub):
        R = L.sub_dofs[i].size
        k = 0 if L.subs[i]["type"] == "stokes" else int(g2l[l, L.subs[i]["region"]])
        S_loc.append(ctx.get_basis(i, k, R))
    return itf.assemble(L, S_loc)


@pytest.mark.parametrize("name", ["cfg2", "cfg3"])
def test_interface_residual_full_size(name):
    print("case: CG residual property", name, flush=True)
    prob = problem(name)
    L = Layout(prob)
    ctx = gpu_ctx(prob, "fp64")
    sz = ctx.sizes()
    n, nr = sz["n_real"], sz["n_region"]
    g2l = ctx.index_map("g2l").reshape(n, nr)
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(n, 24, replace=False))
    g, lam, it, rr, st, rc = gpu_solve(ctx, idx, rtol=1e-8)
    assert (st == 0).all() and (rr <= 1e-8).all()
    gH, G = ctx.interface_data()
    assert G.shape[0] == sz["n_kernel"]
    if G.shape[0]:
        Q = np.linalg.solve(G @ G.T, G)

        def proj(v):
            return v - G.T @ (Q @ v)
    else:
        def proj(v):
            return v
    lam = lam.cpu().numpy()
    for q, l in enumerate(idx):
        S = _assembled_S(ctx, L, g2l, l)
        r = proj(gH - S @ lam[q])
        assert np.linalg.norm(r) <= 2e-8 * np.linalg.norm(proj(gH)), (name, l)
        if G.shape[0]:
            assert np.abs(G @ lam[q]).max() <= 1e-10 * np.abs(G).max() * np.abs(lam[q]).max()
    ctx.close()


def test_lambda_moments_are_weighted_sums_cfg2():
    print("case: cfg2 lambda moments vs weighted sums", flush=True)
    import torch
    ctx = gpu_ctx(problem("cfg2"), "fp64")
    n = ctx.sizes()["n_real"]
    g, lam, it, rr, st, rc = gpu_solve(ctx, np.arange(n), rtol=1e-8)
    assert (st == 0).all()
    ctx.accumulate_moments(g, lam)
    torch.cuda.synchronize()
    _, w = ctx.collocation()
    lam = lam.cpu().numpy()
    mean = w @ lam
    m2 = w @ (lam * lam)
    mg, vg = ctx.get_moments("lambda")
    assert rel(mg, mean) < 1e-12
    assert np.abs(vg - (m2 - mean ** 2)).max() < 1e-12 * np.abs(m2).max()
    ctx.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 0.0), ("mixed", 1e-10)])
def test_basis_layouts_agree_on_the_uneven_layout(precision, tol):
    """The Darcy units of the uneven layout through one launch per shape class,
    one launch per phase over the whole cost-sorted queue, and the tuned
    choice (Section 5.4 pre-computation loop): the same S for one unit of
    every mesh shape, bit for bit in FP64 (every right-hand side is swept by
    the same per-column arithmetic), to the refinement tolerance in mixed
    precision (each group of right-hand sides is refined on its own)."""
    print("case: Darcy basis layouts on the uneven layout", precision, flush=True)
    import torch  # noqa: F401
    from paper_1802_06263_amd import sdmm
    prob = problem("cfg3")
    L = Layout(prob)
    grid = Grid(prob["regions"], prob["rule"])
    units = sampled_units(L, grid, "cfg3", np.random.default_rng(5))
    got = {}
    for mode in (1, 2, 0):
        ctx = sdmm.Context(0)
        ctx.set_problem(prob)
        ctx.set_option("basis_launch", mode)
        ctx.build_flux_basis(precision)
        if mode == 0:
            ctx.build_flux_basis(precision)   # the second build uses the tuned choice
        got[mode] = [ctx.get_basis(i, k, L.sub_dofs[i].size) for i, k in units]
        ctx.close()
    for mode in (2, 0):
        for (i, k), a, b in zip(units, got[1], got[mode]):
            if tol == 0.0:
                assert np.array_equal(a, b), (mode, i, k)
            else:
                assert rel(b, a) < tol, (mode, i, k, rel(b, a))


def test_autotune_keeps_results():
    print("case: autotune on the small FETI case", flush=True)
    prob = problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})
    ctx = gpu_ctx(prob, "fp64")
    n = ctx.sizes()["n_real"]
    g, lam0, it0, _, st0, _ = gpu_solve(ctx, np.arange(n), rtol=1e-10)
    c0 = ctx.counters()
    chunk = ctx.autotune(g, rtol=1e-10)
    ns = min(n, 16384)
    assert 1 <= chunk <= ns
    c1 = ctx.counters()
    assert c1["cg_iterations"] == c0["cg_iterations"]
    _, lam1, it1, _, st1, _ = gpu_solve(ctx, np.arange(n), rtol=1e-10)
    assert np.array_equal(lam0.cpu().numpy(), lam1.cpu().numpy())
    assert np.array_equal(it0, it1) and np.array_equal(st0, st1)
    ctx.close()


CG_CONVERGED, CG_MAXITER = 0, 1   # status values of sdmm_solve_interface


def test_cg_slot_refill_keeps_results():
    """The CG keeps a fixed number of realizations in flight and starts a
    pending realization in each finished one's slot.  Every output must be
    bit-identical whatever the slot count, also for realizations that stop at
    max_iter, and the iteration counter must add up the same."""
    print("case: CG slot refill on cfg1", flush=True)
    ctx = gpu_ctx(problem("cfg1"), "fp64")
    n = ctx.sizes()["n_real"]
    idx = np.arange(n)[::-1].copy()   # slots then hold non-consecutive global indices
    ctx.set_option("cg_chunk", n)
    c0 = ctx.counters()["cg_iterations"]
    _, lam_r, it_r, rr_r, st_r, _ = gpu_solve(ctx, idx, rtol=1e-10)
    tot_r = ctx.counters()["cg_iterations"] - c0
    assert (st_r == CG_CONVERGED).all() and tot_r == int(it_r.sum())
    for slots, lanes in ((n, 1), (50, 2), (3, 2)):
        print("case: cfg1 with %d CG slots, lanes option %d" % (slots, lanes), flush=True)
        ctx.set_option("cg_chunk", slots)
        ctx.set_option("cg_lanes", lanes)
        c0 = ctx.counters()["cg_iterations"]
        _, lam, it, rr, st, _ = gpu_solve(ctx, idx, rtol=1e-10)
        assert ctx.counters()["cg_iterations"] - c0 == tot_r
        assert np.array_equal(lam.cpu().numpy(), lam_r.cpu().numpy())
        assert np.array_equal(it, it_r) and np.array_equal(rr, rr_r) and np.array_equal(st, st_r)
    print("case: cfg1 stopped at max_iter with 7 and 361 slots", flush=True)
    out = []
    ctx.set_option("cg_lanes", 2)
    for slots in (7, n):
        ctx.set_option("cg_chunk", slots)
        _, lam, it, rr, st, _ = gpu_solve(ctx, idx, rtol=1e-10, max_iter=40, allow_notconv=True)
        out.append((lam.cpu().numpy(), it, rr, st))
    assert (out[0][3] == CG_MAXITER).all() and (out[0][1] == 40).all()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    ctx.close()


def test_cg_two_lanes_keep_results():
    """From 2048 slots the CG runs two lanes on two streams whose kernels
    overlap; the outputs must be bit-identical to one lane."""
    print("case: cfg2 with 4096 slots, two lanes against one", flush=True)
    ctx = gpu_ctx(problem("cfg2"), "fp64")
    n = ctx.sizes()["n_real"]
    idx = np.arange(n)
    ctx.set_option("cg_chunk", 4096)
    out = []
    for lanes in (2, 1):
        ctx.set_option("cg_lanes", lanes)
        c0 = ctx.counters()["cg_iterations"]
        _, lam, it, rr, st, _ = gpu_solve(ctx, idx, rtol=1e-8)
        out.append((lam.cpu().numpy(), it, rr, st, ctx.counters()["cg_iterations"] - c0))
    assert (out[0][3] == CG_CONVERGED).all()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    print("case: cfg2 stopped at max_iter, two lanes against one", flush=True)
    out = []
    for lanes in (2, 1):
        ctx.set_option("cg_lanes", lanes)
        _, lam, it, rr, st, _ = gpu_solve(ctx, idx, rtol=1e-8, max_iter=40, allow_notconv=True)
        out.append((lam.cpu().numpy(), it, rr, st))
    assert (out[0][3] == CG_MAXITER).all() and (out[0][1] == 40).all()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    ctx.close()


def test_mixed_moments_match_fp64_cfg2():
    """Full-size precision property on the 6561-realization layout: the whole
    mixed-precision path (FP32 factor, FP64-refined responses, then CG and
    moments) gives the moments of the FP64 path to 1e-8 relative in every
    field.  The FP64 path itself is checked against the oracle on the smaller
    layouts.  The CG runs to rtol 1e-12 so that the comparison measures the
    basis, not the stopping."""
    print("case: cfg2 moments, mixed against FP64", flush=True)
    from paper_1802_06263_amd.sdmm import FIELDS as SFIELDS
    mom = {}
    for prec in ("fp64", "mixed"):
        ctx = gpu_ctx(problem("cfg2"), prec)
        n = ctx.sizes()["n_real"]
        g, lam, it, rr, st, _ = gpu_solve(ctx, np.arange(n), rtol=1e-12)
        assert (st == CG_CONVERGED).all()
        ctx.accumulate_moments(g, lam)
        mom[prec] = {f: ctx.get_moments(f) for f in SFIELDS}
        if prec == "mixed":
            assert ctx.counters()["max_refine_residual"] <= 1e-11
        ctx.close()
    for f in SFIELDS:
        (m64, v64), (mmx, vmx) = mom["fp64"][f], mom["mixed"][f]
        em, ev = rel(mmx, m64), rel(vmx, v64)
        print("  %s: mean %.2e, variance %.2e" % (f, em, ev), flush=True)
        assert em < 1e-8 and ev < 1e-8, f


def test_mixed_basis_moments_match_fp64_cfg3():
    """The same property for the bases of the uneven layout (54273
    realizations), with the interface solution held fixed: both contexts
    accumulate the moments of one FP64 CG solution, so the comparison sees
    only the bases and fine responses.  (Through the whole path the CG
    stopping dominates there: the FP64 moments of lambda at rtol 1e-10 and
    1e-11 differ by 5e-7.)"""
    print("case: cfg3 moments of one interface solution, mixed against FP64 basis", flush=True)
    from paper_1802_06263_amd.sdmm import FIELDS as SFIELDS
    ctxs = {prec: gpu_ctx(problem("cfg3"), prec) for prec in ("fp64", "mixed")}
    assert ctxs["mixed"].counters()["max_refine_residual"] <= 1e-11
    n = ctxs["fp64"].sizes()["n_real"]
    g, lam, it, rr, st, _ = gpu_solve(ctxs["fp64"], np.arange(n), rtol=1e-8)
    assert (st == CG_CONVERGED).all()
    mom = {}
    for prec, ctx in ctxs.items():
        ctx.accumulate_moments(g, lam)
        mom[prec] = {f: ctx.get_moments(f) for f in SFIELDS}
        ctx.close()
    for f in SFIELDS:
        (m64, v64), (mmx, vmx) = mom["fp64"][f], mom["mixed"][f]
        em, ev = rel(mmx, m64), rel(vmx, v64)
        print("  %s: mean %.2e, variance %.2e" % (f, em, ev), flush=True)
        assert em < 1e-8 and ev < 1e-8, f
