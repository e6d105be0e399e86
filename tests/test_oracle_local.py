"""Pins of the oracle's subdomain solvers (Section 3.2, Section 5.1)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.darcy import DarcyLocal
from oracle.geometry import Layout
from oracle.stokes import StokesLocal, element_matrices
from workloads import problem


def _interior_darcy(n=16):
    """cfg1 layout: Darcy subdomain 9 sits in the interior (four Darcy-Darcy sides)."""
    L = Layout(problem("cfg1", darcy_mesh=(n, n), stokes_mesh=(8, 8)))
    i = 4 + 5  # Darcy subdomain (1, 1) of the 4x4 block
    assert all(not L.side_is_outer(i, s) for s in ("left", "right", "bottom", "top"))
    return L, i


def _solve_with_edge_data(dl, pfun):
    """Solve the CCFD system with exact Dirichlet averages on every boundary edge."""
    rhs = np.zeros(dl.N)
    for be in dl.bedges:
        t = np.linspace(be["t0"], be["t1"], 7)
        if be["side"] in ("bottom", "top"):
            y = dl.layout.subs[dl.i]["rect"][2 if be["side"] == "bottom" else 3]
            vals = pfun(t, np.full_like(t, y))
        else:
            x = dl.layout.subs[dl.i]["rect"][0 if be["side"] == "left" else 1]
            vals = pfun(np.full_like(t, x), t)
        # Simpson on 7 points is exact for the smooth data to the accuracy needed
        h = (be["t1"] - be["t0"]) / 6
        avg = h / 3 * (vals[0] + 4 * vals[1:-1:2].sum() + 2 * vals[2:-1:2].sum() + vals[-1]) / (be["t1"] - be["t0"])
        rhs[be["cell"]] += be["T"] * avg
    return dl.lu().solve(rhs)


def test_darcy_manufactured_second_order():
    """Harmonic p = e^x sin(y), K = 1: cell-centre pressure error O(h^2)."""
    errs = []
    for n in (8, 16, 32):
        L, i = _interior_darcy(n)
        dl = DarcyLocal(L, i, np.ones(n * n))
        p = _solve_with_edge_data(dl, lambda x, y: np.exp(x) * np.sin(y))
        x0, x1, y0, y1 = L.subs[i]["rect"]
        h = (x1 - x0) / n
        X, Y = np.meshgrid(x0 + (np.arange(n) + 0.5) * h, y0 + (np.arange(n) + 0.5) * h)
        errs.append(np.abs(p - np.exp(X.ravel()) * np.sin(Y.ravel())).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.2), rates


def test_darcy_harmonic_averaging_exact_in_layers():
    """K varying in y only, p = 0 / 1 at bottom / top, no side flux: the exact
    discrete solution is the series-resistance one, i.e. harmonic averaging."""
    L, i = _interior_darcy(8)
    n = 8
    Ky = np.exp(np.linspace(-1.5, 2.0, n))
    K = np.repeat(Ky, n)
    dl = DarcyLocal(L, i, K)
    rhs = np.zeros(dl.N)
    P = dl.P.tolil()
    for be in dl.bedges:
        if be["side"] == "top":
            rhs[be["cell"]] += be["T"] * 1.0
        elif be["side"] in ("left", "right"):
            P[be["cell"], be["cell"]] -= be["T"]  # turn the sides into no-flow
    p = spla.spsolve(P.tocsc(), rhs).reshape(n, n)
    hy = L.subs[i]["h"][1]
    res = np.concatenate([[hy / 2 / Ky[0]], hy / 2 / Ky[:-1] + hy / 2 / Ky[1:], [hy / 2 / Ky[-1]]])
    flux = 1.0 / res.sum()
    expect = np.cumsum(res)[:-1] * flux
    assert np.allclose(p, expect[:, None], rtol=1e-13, atol=1e-14)


def test_darcy_conservation_and_spd_basis():
    L, i = _interior_darcy(16)
    rng = np.random.default_rng(1)
    K = np.exp(rng.standard_normal(256))
    dl = DarcyLocal(L, i, K)
    lam = rng.standard_normal(dl.R)
    p, uout = dl.solve(lam)
    # cell-wise conservation: sum of outgoing fluxes of every cell is zero (q = 0)
    div = np.zeros(dl.N)
    for e, a, b, T in dl.int_edges:
        div[a] += T * (p[a] - p[b])
        div[b] -= T * (p[a] - p[b])
    for k, be in enumerate(dl.medges):
        div[be["cell"]] += uout[k]
    assert np.abs(div).max() < 1e-12 * np.abs(uout).max()
    S = dl.basis()
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    # an interior Darcy subdomain has no outer pressure data: a constant
    # interface pressure drives no flux, so S is PSD with the constants as kernel
    assert np.abs(S @ np.ones(dl.R)).max() < 1e-12 * np.abs(S).max()
    assert ev[0] > -1e-13 * ev[-1] and ev[1] > 1e-6 * ev[-1]


def test_stokes_element_manufactured_rates():
    """psi = x e^x sin y is biharmonic; u = (psi_y, -psi_x), p = 2 e^x cos y
    solve Stokes with f = 0 (nu = 1).
    Dirichlet velocity on the whole boundary, mean-zero pressure: the Q2-Q1
    velocity error is O(h^3) at nodes and the pressure error O(h^2)."""
    eu, ep = [], []
    for n in (4, 8, 16):
        h = 1.0 / n
        Ae, Be = element_matrices(h, h, 1.0)
        nn = 2 * n + 1
        nv, npr = 2 * nn * nn, (n + 1) ** 2
        rows, cols, vals, br, bc, bv = [], [], [], [], [], []
        for ey in range(n):
            for ex in range(n):
                nodes = [(2 * ey + b) * nn + 2 * ex + a for b in range(3) for a in range(3)]
                d = np.array([[2 * q, 2 * q + 1] for q in nodes]).ravel()
                pn = np.array([(ey + b) * (n + 1) + ex + a for b in range(2) for a in range(2)])
                r, c = np.meshgrid(d, d, indexing="ij")
                rows += [r.ravel()]; cols += [c.ravel()]; vals += [Ae.ravel()]
                r, c = np.meshgrid(pn, d, indexing="ij")
                br += [r.ravel()]; bc += [c.ravel()]; bv += [Be.ravel()]
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), (nv, nv)).tocsr()
        B = sp.coo_matrix((np.concatenate(bv), (np.concatenate(br), np.concatenate(bc))), (npr, nv)).tocsr()
        X, Y = np.meshgrid(np.linspace(0, 1, nn), np.linspace(0, 1, nn))
        ue = np.zeros(nv)
        ue[0::2] = (X * np.exp(X) * np.cos(Y)).ravel()
        ue[1::2] = (-(1 + X) * np.exp(X) * np.sin(Y)).ravel()
        bnd = (X.ravel() == 0) | (X.ravel() == 1) | (Y.ravel() == 0) | (Y.ravel() == 1)
        dd = np.nonzero(bnd)[0]
        dir_dofs = np.sort(np.concatenate([2 * dd, 2 * dd + 1]))
        fr = np.setdiff1d(np.arange(nv), dir_dofs)
        uD = np.zeros(nv)
        uD[dir_dofs] = ue[dir_dofs]
        Xp, Yp = np.meshgrid(np.linspace(0, 1, n + 1), np.linspace(0, 1, n + 1))
        pe = (2 * np.exp(Xp) * np.cos(Yp)).ravel()
        mass1 = np.full(npr, h * h)  # constant-pressure constraint row (weights only fix the constant)
        K = sp.bmat([[A[fr][:, fr], B[:, fr].T, None], [B[:, fr], None, sp.csr_matrix(mass1[:, None])],
                     [None, sp.csr_matrix(mass1[None, :]), None]], format="csc")
        rhs = np.concatenate([-(A @ uD)[fr], -(B @ uD), [mass1 @ pe]])
        x = spla.splu(K).solve(rhs)
        u = uD.copy()
        u[fr] = x[:fr.size]
        p = x[fr.size:fr.size + npr]
        eu.append(np.abs(u - ue).max())
        ep.append(np.abs(p - pe).max())
    ru = np.log2(np.array(eu[:-1]) / np.array(eu[1:]))
    rp = np.log2(np.array(ep[:-1]) / np.array(ep[1:]))
    assert eu[0] > 1e-8 and np.all(ru > 2.8), (eu, ru)
    assert np.all(rp > 1.8), rp


def test_stokes_local_operators():
    L = Layout(problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2}))
    seen_float = False
    for i in range(L.n_stokes):
        st = StokesLocal(L, i)
        S = st.basis()
        assert np.abs(S - S.T).max() <= 1e-10 * np.abs(S).max()
        ev = np.linalg.eigvalsh(0.5 * (S + S.T))
        if st.floating:
            seen_float = True
            assert st.Z.shape[1] == 2
            assert np.abs(st.A @ st.Z).max() < 1e-12 and np.abs(st.B @ st.Z).max() < 1e-12
        # a uniform normal stress produces no velocity (div u = 0, and u = 0 on
        # the outer boundary or u orthogonal to the rigid motions), so S is PSD
        # with exactly one null vector
        assert ev[0] > -1e-12 * ev[-1] and ev[1] > 1e-8 * ev[-1]
    assert seen_float
