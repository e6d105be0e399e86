"""Pins of the oracle's exactly integrated RT0 mass in hybridized form (the
Darcy discretization of the paper's numerical cases, Section 6).

* the cell mass against 2-D Gauss quadrature of the RT0 basis functions;
* the monolithic pair mass against quadrature of the 1-D shape functions;
* S1, S2 and S3 against the coupled system solved directly in mixed form
  (Section 4, eqs. fullydisc1-2), which shares no elimination with the
  hybridized face-pressure system;
* second-order cell pressures on a smooth harmonic field, and a result that
  differs from the trapezoidal mass;
* the constant-permeability closed form (linear pressure, uniform flow);
* a symmetric PSD flux basis with the constants as its kernel;
* planted mistakes (the trapezoidal mass in the hybridized cell, a flipped
  face orientation) break the comparison with the monolithic solve.
"""
import numpy as np
import pytest

import oracle.darcy as odarcy
from oracle import monolithic
from oracle.darcy import DarcyLocal, DarcyLocalExact
from oracle.geometry import GL3_W, GL3_X, Layout
from oracle.methods import FIELDS, Oracle
from workloads import problem


def _exact(prob):
    prob = dict(prob)
    prob["discretization"] = {"darcy": "exact"}
    return prob


def _interior(n=8):
    L = Layout(_exact(problem("cfg1", darcy_mesh=(n, n), stokes_mesh=(8, 8))))
    return L, 4 + 5


def test_cell_mass_against_quadrature():
    L, i = _interior(4)
    K = np.full(16, 2.5)
    dl = DarcyLocalExact(L, i, K)
    hx, hy, nu = dl.hx, dl.hy, dl.nu
    q = 0.5 * (1 + GL3_X)
    w = 0.5 * GL3_W
    # outward-flux RT0 basis on [0, hx] x [0, hy] in reference coordinates (s, t)
    def basis(s, t):
        return [np.array([-(1 - s) / hy, 0.0]), np.array([s / hy, 0.0]),
                np.array([0.0, -(1 - t) / hx]), np.array([0.0, t / hx])]
    M = np.zeros((4, 4))
    for a, s in enumerate(q):
        for b, t in enumerate(q):
            ph = basis(s, t)
            for m in range(4):
                for n in range(4):
                    M[m, n] += w[a] * w[b] * hx * hy * nu / 2.5 * ph[m] @ ph[n]
    assert np.allclose(dl.cell_mass_fluxes(0), M, rtol=1e-14, atol=1e-14)


def test_pair_mass_against_quadrature():
    q = 0.5 * (1 + GL3_X)
    w = 0.5 * GL3_W
    sh = np.stack([1 - q, q])
    assert np.allclose(monolithic.rt0_pair_mass(True), (sh * w) @ sh.T, rtol=1e-15)
    # the trapezoidal rule samples the shape functions at the two faces only
    assert np.allclose(monolithic.rt0_pair_mass(False), 0.5 * np.eye(2))


def _mono(o, l):
    y = o.grid.points[l]
    Kd = {i: o.darcy_K(i, o.region_point(y, o.L.subs[i]["region"])) for i in o.darcy_ids}
    return monolithic.solve(o.L, Kd, o.stokes)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def cfg0_exact():
    return Oracle(_exact(problem("cfg0")))


@pytest.mark.parametrize("l", [0, 13])
def test_all_methods_match_monolithic(cfg0_exact, l):
    o = cfg0_exact
    m = _mono(o, l)
    for meth in ("S1", "S2", "S3"):
        f, it, rel, ok = getattr(o, "realization_" + meth)(l, rtol=1e-12)
        assert ok
        for k in FIELDS:
            assert _rel(f[k], m[k]) < 1e-9, (meth, k, _rel(f[k], m[k]))


def test_exact_differs_from_trapezoidal(cfg0_exact):
    f, *_ = cfg0_exact.realization_S3(13, rtol=1e-12)
    g, *_ = Oracle(problem("cfg0")).realization_S3(13, rtol=1e-12)
    assert _rel(f["darcy_p"], g["darcy_p"]) > 1e-4


def test_feti_layout_matches_monolithic():
    o = Oracle(_exact(problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})))
    m = _mono(o, 4000)
    f, it, rel, ok = o.realization_S3(4000, rtol=1e-12)
    assert ok
    for k in FIELDS:
        assert _rel(f[k], m[k]) < 1e-9, k


def _edge_average(L, i, be, pfun):
    t = np.linspace(be["t0"], be["t1"], 7)
    if be["side"] in ("bottom", "top"):
        y = L.subs[i]["rect"][2 if be["side"] == "bottom" else 3]
        vals = pfun(t, np.full_like(t, y))
    else:
        x = L.subs[i]["rect"][0 if be["side"] == "left" else 1]
        vals = pfun(np.full_like(t, x), t)
    h = (be["t1"] - be["t0"]) / 6
    return h / 3 * (vals[0] + 4 * vals[1:-1:2].sum() + 2 * vals[2:-1:2].sum() + vals[-1]) / (be["t1"] - be["t0"])


def test_manufactured_second_order():
    """Harmonic p = e^x sin(y), K = 1, exact edge averages as face pressures
    on the boundary: cell-centre pressure error O(h^2)."""
    pf = lambda x, y: np.exp(x) * np.sin(y)
    errs = []
    for n in (8, 16, 32):
        L, i = _interior(n)
        dl = DarcyLocalExact(L, i, np.ones(n * n))
        mu = np.zeros(dl.ne)
        for be in dl.bedges:
            mu[be["edge"]] = _edge_average(L, i, be, pf)
        mu[dl.unknown] = dl.lu().solve(-(dl.Huk @ mu[dl.known]))
        p, U = dl.cell_fluxes(mu)
        x0, x1, y0, y1 = L.subs[i]["rect"]
        h = (x1 - x0) / n
        X, Y = np.meshgrid(x0 + (np.arange(n) + 0.5) * h, y0 + (np.arange(n) + 0.5) * h)
        errs.append(np.abs(p - pf(X.ravel(), Y.ravel())).max())
        # every cell conserves mass
        assert np.abs(U.sum(axis=1)).max() < 1e-12 * np.abs(U).max()
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.25), (errs, rates)


def test_constant_permeability_closed_form():
    """sigma^2 = 0: u = (0, -1) in both regions and p_d = y are in the RT0-Q0
    spaces for either mass, so the exact-mass path reproduces them."""
    o = Oracle(_exact(problem("cfg0", sigma2=0.0)))
    for meth in ("S1", "S3"):
        f, it, rel, ok = getattr(o, "realization_" + meth)(3, rtol=1e-13)
        assert ok
        yc = (np.arange(8) + 0.5) / 8
        assert np.allclose(f["darcy_p"].reshape(2, 8, 8), yc[None, :, None], atol=1e-11)
        du = f["darcy_u"].reshape(2, -1)
        nv = 9 * 8
        assert np.abs(du[:, :nv]).max() < 1e-11 and np.abs(du[:, nv:] + 1).max() < 1e-11


def test_spd_basis_with_constant_kernel():
    L, i = _interior(16)
    K = np.exp(np.random.default_rng(2).standard_normal(256))
    S = DarcyLocalExact(L, i, K).basis()
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    assert np.abs(S @ np.ones(S.shape[0])).max() < 1e-12 * np.abs(S).max()
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev[0] > -1e-13 * ev[-1] and ev[1] > 1e-6 * ev[-1]
    # not the trapezoidal operator
    Lt = Layout(problem("cfg1", darcy_mesh=(16, 16), stokes_mesh=(8, 8)))
    assert _rel(S, DarcyLocal(Lt, i, K).basis()) > 1e-3


@pytest.mark.parametrize("mistake", ["trapezoidal_cell_mass", "face_orientation"])
def test_monolithic_pin_catches_planted_mistakes(monkeypatch, mistake, cfg0_exact):
    if mistake == "trapezoidal_cell_mass":
        def lumped(self, c):
            M = np.diag(0.5 * self.nu * self.hx * self.hy / self.K[c] / self.face_len ** 2)
            return M
        monkeypatch.setattr(DarcyLocalExact, "cell_mass_fluxes", lumped)
        # the lumped cell mass is right for the trapezoidal path: check the pin
        # sees the difference against the exact-mass monolithic solve
    else:
        orig = DarcyLocalExact.__init__

        def flipped(self, layout, i, K):
            orig(self, layout, i, K)
            self.face_sign = np.array([1.0, 1.0, -1.0, 1.0])
        monkeypatch.setattr(DarcyLocalExact, "__init__", flipped)
    o = Oracle(_exact(problem("cfg0")))
    f, *_ = o.realization_S3(13, rtol=1e-12)
    m = _mono(cfg0_exact, 13)
    assert max(_rel(f[k], m[k]) for k in FIELDS) > 1e-6
