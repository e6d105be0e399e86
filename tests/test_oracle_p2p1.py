"""Pins of the oracle's triangular Taylor-Hood pair (P2-P1), the element of
the paper's numerical cases (Section 6), beside the Q2-Q1 default.

* P2-P1 holds quadratic velocities and linear pressures, so a Stokes
  solution of that form (zero body force) is reproduced to rounding on any
  mesh, here with hx != hy and the corner cuts;
* on a smooth solution the nodal velocity error falls like h^3 and the
  pressure error like h^2;
* planted mistakes (a quadrature rule that is not exact for degree 2, a
  pressure basis tied to the wrong vertex) break the first pin;
* the element changes the operator but none of the index maps, and the
  method's Couette pin over a BJS interface holds with it.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle.stokes as ostokes
from oracle.geometry import Layout
from oracle.methods import Oracle
from oracle.stokes import StokesLocal, diagonal, element_matrices_p2p1
from workloads import problem


def _dirichlet_solve(nx, ny, lx, ly, ufun, pfun, element="p2p1"):
    """Assemble one nx x ny rectangle mesh of [0,lx]x[0,ly], impose the exact
    velocity on the whole boundary and the exact pressure mean; return the
    nodal velocity and pressure errors."""
    hx, hy = lx / nx, ly / ny
    blocks = {d: element_matrices_p2p1(hx, hy, 1.0, d) for d in ("/", "\\")}
    if element == "q2q1":
        blocks = dict.fromkeys(("/", "\\"), ostokes.element_matrices(hx, hy, 1.0))
    nnx, nny = 2 * nx + 1, 2 * ny + 1
    nv, npr = 2 * nnx * nny, (nx + 1) * (ny + 1)
    rows, cols, vals, br, bc, bv = [], [], [], [], [], []
    for ey in range(ny):
        for ex in range(nx):
            Ae, Be = blocks[diagonal(ex, ey, nx, ny)]
            nodes = [(2 * ey + b) * nnx + 2 * ex + a for b in range(3) for a in range(3)]
            d = np.array([[2 * q, 2 * q + 1] for q in nodes]).ravel()
            pn = np.array([(ey + b) * (nx + 1) + ex + a for b in range(2) for a in range(2)])
            r, c = np.meshgrid(d, d, indexing="ij")
            rows += [r.ravel()]; cols += [c.ravel()]; vals += [Ae.ravel()]
            r, c = np.meshgrid(pn, d, indexing="ij")
            br += [r.ravel()]; bc += [c.ravel()]; bv += [Be.ravel()]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), (nv, nv)).tocsr()
    B = sp.coo_matrix((np.concatenate(bv), (np.concatenate(br), np.concatenate(bc))), (npr, nv)).tocsr()
    X, Y = np.meshgrid(np.linspace(0, lx, nnx), np.linspace(0, ly, nny))
    ue = np.zeros(nv)
    ux, uy = ufun(X, Y)
    ue[0::2], ue[1::2] = ux.ravel(), uy.ravel()
    ib = np.nonzero((np.abs(X.ravel()) < 1e-14) | (np.abs(X.ravel() - lx) < 1e-14)
                    | (np.abs(Y.ravel()) < 1e-14) | (np.abs(Y.ravel() - ly) < 1e-14))[0]
    dd = np.sort(np.concatenate([2 * ib, 2 * ib + 1]))
    fr = np.setdiff1d(np.arange(nv), dd)
    uD = np.zeros(nv)
    uD[dd] = ue[dd]
    Xp, Yp = np.meshgrid(np.linspace(0, lx, nx + 1), np.linspace(0, ly, ny + 1))
    pe = pfun(Xp, Yp).ravel()
    one = np.ones(npr)
    K = sp.bmat([[A[fr][:, fr], B[:, fr].T, None], [B[:, fr], None, sp.csr_matrix(one[:, None])],
                 [None, sp.csr_matrix(one[None, :]), None]], format="csc")
    rhs = np.concatenate([-(A @ uD)[fr], -(B @ uD), [one @ pe]])
    x = spla.splu(K).solve(rhs)
    u = uD.copy()
    u[fr] = x[:fr.size]
    p = x[fr.size:fr.size + npr]
    return np.abs(u - ue).max(), np.abs(p - pe).max(), np.abs(ue).max()


_POLY = [
    # u = (x^2, -2xy): div u = 0, -lap u + grad p = 0 with p = 2x
    (lambda X, Y: (X * X, -2 * X * Y), lambda X, Y: 2 * X),
    # u = (x^2 - y^2, -2xy) is harmonic and divergence-free, p = 0
    (lambda X, Y: (X * X - Y * Y, -2 * X * Y), lambda X, Y: 0 * X),
    # u = (y^2, 0), p = 2x
    (lambda X, Y: (Y * Y, 0 * X), lambda X, Y: 2 * X),
]


@pytest.mark.parametrize("k", range(len(_POLY)))
def test_p2p1_reproduces_quadratic_stokes_flows(k):
    uf, pf = _POLY[k]
    eu, ep, us = _dirichlet_solve(5, 3, 1.0, 0.75, uf, pf)
    assert eu < 1e-12 * max(us, 1.0) and ep < 1e-11, (eu, ep)


def test_p2p1_manufactured_rates():
    """psi = x e^x sin y: u = (psi_y, -psi_x), p = 2 e^x cos y, f = 0, nu = 1."""
    uf = lambda X, Y: (X * np.exp(X) * np.cos(Y), -(1 + X) * np.exp(X) * np.sin(Y))
    pf = lambda X, Y: 2 * np.exp(X) * np.cos(Y)
    eu, ep = [], []
    for n in (4, 8, 16):
        a, b, _ = _dirichlet_solve(n, n, 1.0, 1.0, uf, pf)
        eu.append(a)
        ep.append(b)
    ru = np.log2(np.array(eu[:-1]) / np.array(eu[1:]))
    rp = np.log2(np.array(ep[:-1]) / np.array(ep[1:]))
    assert eu[0] > 1e-8 and np.all(ru > 2.5), (eu, ru)
    assert np.all(rp > 1.5), (ep, rp)


@pytest.mark.parametrize("mistake", ["centroid_rule", "pressure_vertex"])
def test_p2p1_pin_catches_planted_mistakes(monkeypatch, mistake):
    if mistake == "centroid_rule":
        monkeypatch.setattr(ostokes, "_TRI_RULE", (np.array([[1 / 3, 1 / 3, 1 / 3]]), np.ones(1)))
    else:
        monkeypatch.setattr(ostokes, "_pressure_node", lambda a, b: 2 * (a // 2) + b // 2)
    uf, pf = _POLY[0]
    eu, ep, us = _dirichlet_solve(5, 3, 1.0, 0.75, uf, pf)
    assert eu > 1e-6 or ep > 1e-6, (eu, ep)


def _p2p1(prob):
    prob = dict(prob)
    prob["discretization"] = {"stokes": "p2p1"}
    return prob


def test_p2p1_changes_the_operator_not_the_maps():
    small = problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})
    La, Lb = Layout(small), Layout(_p2p1(small))
    for i in range(La.n_stokes):
        a, b = StokesLocal(La, i), StokesLocal(Lb, i)
        assert (a.nvel, a.npre, a.R) == (b.nvel, b.npre, b.R)
        assert np.array_equal(a.free, b.free) and np.array_equal(a.Q, b.Q)
        assert abs(a.A - b.A).max() > 1e-3
        # every node pair the triangles couple is coupled by the rectangles
        # (the band of the operator does not grow)
        nodes = lambda M: {(r // 2, c // 2) for r, c in zip(*M.nonzero())}
        assert nodes(b.A) <= nodes(a.A)
        S = b.basis()
        assert np.abs(S - S.T).max() <= 1e-10 * np.abs(S).max()
        if b.floating:
            assert b.Z.shape[1] == 2 and np.abs(b.A @ b.Z).max() < 1e-12


@pytest.mark.parametrize("l", [0, 13])
def test_p2p1_all_methods_match_monolithic_cfg0(l):
    """The interface reduction with the triangular element against the
    coupled system solved directly (Section 4, eqs. fullydisc1-2)."""
    from oracle import monolithic
    from oracle.methods import FIELDS
    o = Oracle(_p2p1(problem("cfg0")))
    y = o.grid.points[l]
    Kd = {i: o.darcy_K(i, o.region_point(y, o.L.subs[i]["region"])) for i in o.darcy_ids}
    m = monolithic.solve(o.L, Kd, o.stokes)
    for meth in ("S1", "S2", "S3"):
        f, it, rel, ok = getattr(o, "realization_" + meth)(l, rtol=1e-12)
        assert ok
        for k in FIELDS:
            d = np.abs(f[k] - m[k]).max() / max(np.abs(m[k]).max(), 1e-300)
            assert d < 1e-9, (meth, k, d)
