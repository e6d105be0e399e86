"""The full-size 4x2 Stokes over 8x4 Darcy layout against stored oracle values (needs an MI355X).

tests/golden/cfg2_reference.npz is written by tests/golden/make_cfg2_reference.py,
which calls only the FP64 oracle.  Compared element by element:

  * every Stokes S_{H,i} (eqs. starSproblem1-2; the two floating subdomains
    included), g_H (eqs. barSproblem1-2) and the range of the FETI matrix G
    (its rows may be any orthonormal basis of the rigid-motion traces): 1e-10
    relative, with no FP64 refinement step after the band LDL^T (the
    default) and with two.  Both sides solve the 64x64 Taylor-Hood saddle
    systems to a relative residual near 1e-14 (sparse LU with one refinement
    step on the oracle's side), so they differ by the forward error the
    conditioning allows: the 1-norm condition estimate of these systems is
    about 2.4e7, i.e. a worst case of about 3e-9 relative; the observed
    differences are near 1e-11;
  * lambda of 24 seeded collocation points at CG rtol 1e-12: 1e-9 (FP64),
    1e-8 (mixed) relative (CG stopping error times the interface condition
    number);
  * the weighted means and variances (Section 2) of all five fields over
    those 24 points, on the stored sample of entries of each field, relative
    to the largest |mean| / |var| of the whole field: 1e-9 (FP64), 1e-8 (mixed).
"""
import os

import numpy as np
import pytest

from oracle.methods import FIELDS
from workloads import problem

from gpu_helpers import gpu_ctx, gpu_solve, rel

pytestmark = pytest.mark.gpu

REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg2_reference.npz")


def _range_projector(G):
    """G^T (G G^T)^{-1} G for G with one row per rigid-motion mode (n_kernel x M)."""
    return G.T @ np.linalg.solve(G @ G.T, G)


@pytest.fixture(scope="module")
def ref():
    return dict(np.load(REF, allow_pickle=False))


@pytest.mark.parametrize("refine", [0, 2])
def test_stokes_bases_and_interface_data(ref, refine):
    print("case: cfg2 Stokes bases, g_H and G vs stored oracle values, refinement steps", refine, flush=True)
    import torch  # noqa: F401
    from paper_1802_06263_amd import sdmm
    ctx = sdmm.Context(0)
    ctx.set_problem(problem("cfg2"))
    ctx.set_option("stokes_refine", refine)
    ctx.build_flux_basis("fp64")
    errs = {}
    for i in ref["stokes_ids"]:
        S = ref["S_stokes_%d" % i]
        errs["S_%d" % i] = rel(ctx.get_basis(int(i), 0, S.shape[0]), S)
    g, G = ctx.interface_data()
    errs["g_H"] = rel(g, ref["g"])
    assert G.shape == ref["G"].shape
    # a floating subdomain's rigid motions may be any orthonormal basis of the
    # same 2-dimensional space, so G is compared through the projector onto
    # its range, the only way the FETI projection and recovery use it
    errs["G_range"] = rel(_range_projector(G), _range_projector(ref["G"]))
    print("  " + " ".join("%s %.2e" % kv for kv in errs.items()), flush=True)
    for k, e in errs.items():
        assert e < 1e-10, (k, e)
    ctx.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-8)])
def test_lambda_and_moments_vs_stored_oracle(ref, precision, tol):
    print("case: cfg2 lambda and moments of 24 points vs stored oracle values", precision, flush=True)
    import torch
    ctx = gpu_ctx(problem("cfg2"), precision)
    idx = ref["idx"]
    g, lam, it, rr, st, rc = gpu_solve(ctx, idx, rtol=float(ref["rtol"]))
    assert (st == 0).all()
    assert rel(lam.cpu().numpy(), ref["lambda"]) < tol
    ctx.reset_moments()
    ctx.accumulate_moments(g, lam, torch.tensor(ref["weights"], device="cuda"))
    for f in FIELDS:
        mg, vg = ctx.get_moments(f)
        assert mg.size == int(ref["size_" + f]), f
        sel = ref["sel_" + f]
        mo, vo = ref["mean_" + f], ref["var_" + f]
        em = np.abs(mg[sel] - mo).max() / float(ref["maxmean_" + f])
        ev = np.abs(vg[sel] - vo).max() / max(float(ref["maxvar_" + f]), 1e-12 * float(ref["maxmean_" + f]) ** 2)
        print("  %s %s mean %.2e var %.2e" % (precision, f, em, ev), flush=True)
        assert em < tol, (f, em)
        assert ev < tol, (f, ev)
    ctx.close()
