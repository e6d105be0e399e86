"""Pins of the oracle's interface reduction and Methods S1, S2, S3 (Section 5)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import interface as itf
from oracle import monolithic
from oracle.methods import FIELDS, Oracle
from workloads import problem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _mono(o, l):
    y = o.grid.points[l]
    Kd = {i: o.darcy_K(i, o.region_point(y, o.L.subs[i]["region"])) for i in o.darcy_ids}
    return monolithic.solve(o.L, Kd, o.stokes)


def test_constant_permeability_closed_form():
    """sigma^2 = 0: K = 1 everywhere; u = (0, -1) in both regions, p_d = y,
    p_s = 1 and lambda = the interface pressure, all exactly in the discrete
    spaces, so every method and the monolithic solve reproduce them."""
    o = Oracle(problem("cfg0", sigma2=0.0))
    for meth in ("S1", "S2", "S3"):
        f, it, rel, ok = getattr(o, "realization_" + meth)(3, rtol=1e-13)
        assert ok
        su = f["stokes_u"]
        assert np.abs(su[0::2]).max() < 1e-11 and np.abs(su[1::2] + 1).max() < 1e-11
        assert np.abs(f["stokes_p"] - 1.0).max() < 1e-9
        ny = 8
        yc = (np.arange(ny) + 0.5) / ny
        assert np.allclose(f["darcy_p"].reshape(2, ny, 8), yc[None, :, None], atol=1e-11)
        du = f["darcy_u"].reshape(2, -1)
        nv = 9 * 8
        assert np.abs(du[:, :nv]).max() < 1e-11 and np.abs(du[:, nv:] + 1).max() < 1e-11
    lam = f["lambda"]
    L = o.L
    for fa in L.ifaces:
        if fa.kind == "sd":
            assert np.allclose(lam[fa.off:fa.off + fa.ndof], 1.0, atol=1e-11)
        if fa.kind == "dd":  # vertical interface x = 0.5: lambda = y at the P1 nodes
            t = np.array([fa.a + (e + s) * fa.H for e in range(fa.nelem) for s in (0, 1)])
            assert np.allclose(lam[fa.off:fa.off + fa.ndof], t, atol=1e-11)


@pytest.mark.parametrize("l", [0, 7, 13])
def test_all_methods_match_monolithic_cfg0(cfg0_oracle, l):
    o = cfg0_oracle
    m = _mono(o, l)
    for meth in ("S1", "S2", "S3"):
        f, it, rel, ok = getattr(o, "realization_" + meth)(l, rtol=1e-12)
        assert ok
        for k in FIELDS:
            assert _rel(f[k], m[k]) < 1e-9, (meth, k)


def test_feti_floating_stokes_matches_monolithic():
    p = problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})
    o = Oracle(p)
    assert o.G.shape[1] == 4
    for l in (0, 4000):
        m = _mono(o, l)
        f, it, rel, ok = o.realization_S3(l, rtol=1e-12)
        assert ok
        for k in FIELDS:
            assert _rel(f[k], m[k]) < 1e-9, k


def test_brute_force_schur_equals_assembled_interface_operator():
    """Eliminating every subdomain unknown from the monolithic matrix gives
    S_H = sum_i R_i^T S_{H,i} R_i (eq. operatorform)."""
    o = Oracle(problem("cfg0"))
    l = 9
    y = o.grid.points[l]
    Kd = {i: o.darcy_K(i, o.region_point(y, o.L.subs[i]["region"])) for i in o.darcy_ids}
    Bd, Qall, rhs, _ = monolithic.system(o.L, Kd, o.stokes)
    X = spla.splu(Bd.tocsc()).solve(Qall.T.toarray())
    S_brute = Qall @ X
    S_loc = [None] * o.L.nsub
    for i in o.darcy_ids:
        S_loc[i] = o.darcy_local(i, y).basis()
    for i in o.stokes_ids:
        S_loc[i] = o.stokes[i].basis()
    S = itf.assemble(o.L, S_loc)
    assert _rel(S, S_brute) < 1e-11


def test_S2_and_S3_bases_agree_for_the_same_local_field(cfg0_oracle):
    o = cfg0_oracle
    o.stochastic_basis()
    for l in (0, 5, 15):
        y = o.grid.points[l]
        for i in o.darcy_ids:
            r = o.L.subs[i]["region"]
            k = int(o.grid.g2l[l, r])
            assert _rel(o.darcy_local(i, y).basis(), o.s3_table[(i, k)]) < 1e-13


def test_solve_counters_follow_the_cost_formulas():
    gold = json.load(open(os.path.join(GOLD, "paper_counts.json")))
    for c in gold["cases"]:
        assert (c["ndof"] + 2) * c["nreal"] == c["S2"]
        assert c["ndof"] * c["nreal_local"] + 2 * c["nreal"] == c["S3"]
    o = Oracle(problem("cfg0"))
    L = o.L
    for meth in ("S2", "S3", "S1"):
        mom, info = o.run(meth, rtol=1e-8)
        for i in range(L.nsub):
            R = L.sub_dofs[i].size
            if meth == "S2":
                assert o.counters[i] == (R + 2) * o.grid.nreal
            elif meth == "S3":
                Lj = o.grid.nlocal[L.subs[i]["region"]] if L.subs[i]["type"] == "darcy" else 1
                assert o.counters[i] == R * Lj + 2 * o.grid.nreal
            else:
                assert o.counters[i] == sum(d["iters"] + 2 for d in info)


def test_zero_variance_when_sigma_is_zero():
    o = Oracle(problem("cfg0", sigma2=0.0))
    mom, info = o.run("S3", rtol=1e-12)
    f, *_ = o.realization_S3(0, rtol=1e-12)
    for k in FIELDS:
        mean, var = mom[k]
        assert np.abs(var).max() < 1e-12 * max(1.0, np.abs(mean).max() ** 2)
        assert np.abs(mean - f[k]).max() < 1e-12 * max(1.0, np.abs(f[k]).max())


def test_moments_are_weighted_sums(cfg0_oracle):
    """E and Var = E[u^2] - E[u]^2 with the collocation weights (Sections 2, 4)."""
    o = cfg0_oracle
    idx = [0, 3, 8]
    w = np.array([0.2, 0.5, 0.3])
    mom, info = o.run("S3", indices=idx, weights=w, rtol=1e-12)
    lam = np.stack([d["lambda"] for d in info])
    assert np.allclose(mom["lambda"][0], w @ lam, rtol=1e-14, atol=1e-15)
    assert np.allclose(mom["lambda"][1], w @ lam ** 2 - (w @ lam) ** 2, rtol=1e-12, atol=1e-14)


def test_closed_form_stokes_pressure_on_the_cfg1_meshes():
    """sigma^2 = 0 on the cfg1 layout (Stokes 32x32 Q2-Q1): p_s = 1 and
    u = (0, -1) exactly in the discrete spaces.  The saddle solves must reach
    the discrete solution to near machine precision: with one refinement
    step after the sparse LU the pressure error is about 1e-11 (from the CG
    tolerance); without it, about 1e-9."""
    o = Oracle(problem("cfg1", sigma2=0.0))
    f, it, rel, ok = o.realization_S2(0, rtol=1e-13)
    assert ok
    assert np.abs(f["stokes_p"] - 1.0).max() < 1e-10
    su = f["stokes_u"]
    assert np.abs(su[0::2]).max() < 1e-11 and np.abs(su[1::2] + 1).max() < 1e-11
