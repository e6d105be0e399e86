"""Pins of the oracle parts that the constant-permeability closed form cannot
reach: the BJS slip term, the Stokes mortar coupling under non-constant
data, P2 mortars on non-matching Darcy grids, and the interface reduction on
a non-matching P2 layout.

* Couette flow over a BJS interface (Section 2, eq. BJS; Section 3.2, the
  forms a~_i with the BJS term and b~_Lambda).  With the outer Stokes
  velocity u = (s0 + c (y - 1), 0) and p_d = 0 at y = 0, the coupled problem
  has the exact solution u_s = (s0 + c (y - 1), 0), p_s = 0, p_d = 0,
  u_d = 0, provided the BJS condition holds at y = 1:
      -(sigma n) . tau = nu c = (nu alpha / sqrt(K)) s0,  i.e. s0 = c sqrt(K) / alpha.
  Every field lies in the discrete spaces, so each method reproduces it to
  the CG tolerance.  The Stokes-Stokes mortar then carries the stress
  vector: on a vertical interface -sigma n_i = (0, -nu c), on a horizontal one
  (-nu c, 0) (n_i the outward normal of the lower-numbered subdomain).
* Mortar coupling with non-constant data: the trace operators Q (Stokes) and
  the edge averages (Darcy) against adaptive quadrature of the mortar
  function times a polynomial trace, the mortar basis written here from its
  Lagrange nodes.
* sigma^2 = 0 on a layout with P2 mortars and non-matching Darcy meshes: u =
  (0, -1), p_d = y, p_s = 1; lambda is the trace of the pressure, known at
  every P2 node.
* S1, S2 and S3 against the monolithic solve (eqs. fullydisc1-2) on a tiny
  non-matching P2 layout with a random permeability.

Each pin is shown to fail on a planted mistake in the oracle.
"""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle.geometry as geom
import oracle.stokes as ostokes
from oracle import monolithic
from oracle.geometry import Layout
from oracle.methods import FIELDS, Oracle
from oracle.stokes import StokesLocal
from workloads import problem

ALPHA, NU_S, K_BJS, SHEAR = 0.7, 1.3, 4.0, 0.8
S0 = SHEAR * np.sqrt(K_BJS) / ALPHA   # slip velocity at y = 1 fixed by BJS


def _couette(name, **kw):
    p = problem(name, **kw)
    p["physics"].update({"alpha": ALPHA, "nu_s": NU_S, "k_bjs": K_BJS,
                         "inflow": [S0 - SHEAR, 0.0], "inflow_shear": SHEAR})
    return p


def _stokes_node_y(o):
    ys = []
    for i in o.stokes_ids:
        st = o.stokes[i]
        y0 = o.L.subs[i]["rect"][2]
        y = y0 + 0.5 * st.hy * np.arange(st.nny)
        ys.append(np.repeat(y, st.nnx))
    return np.concatenate(ys)


def _couette_error(o, f):
    """Largest deviation of one realization's fields from the Couette solution."""
    y = _stokes_node_y(o)
    su = f["stokes_u"]
    err = max(np.abs(su[0::2] - (S0 + SHEAR * (y - 1.0))).max(), np.abs(su[1::2]).max(),
              np.abs(f["stokes_p"]).max(), np.abs(f["darcy_p"]).max(), np.abs(f["darcy_u"]).max())
    lam = f["lambda"]
    for fa in o.L.ifaces:
        v = lam[fa.off:fa.off + fa.ndof]
        if fa.kind == "ss":
            want = np.array([0.0, -NU_S * SHEAR]) if fa.orient == "v" else np.array([-NU_S * SHEAR, 0.0])
            err = max(err, np.abs(v.reshape(-1, 2) - want[None, :]).max())
        else:
            err = max(err, np.abs(v).max())
    return err


@pytest.mark.parametrize("element", ["q2q1", "p2p1"])
def test_couette_over_bjs_interface_all_methods_and_monolithic(element):
    p = _couette("cfg0")
    p["discretization"] = {"stokes": element}
    o = Oracle(p)
    for meth in ("S1", "S2", "S3"):
        f, it, rel, ok = getattr(o, "realization_" + meth)(5, rtol=1e-13)
        assert ok
        assert _couette_error(o, f) < 1e-10, meth
    y = o.grid.points[5]
    Kd = {i: o.darcy_K(i, o.region_point(y, o.L.subs[i]["region"])) for i in o.darcy_ids}
    m = monolithic.solve(o.L, Kd, o.stokes)
    assert _couette_error(o, m) < 1e-10


@pytest.mark.parametrize("element", ["q2q1", "p2p1"])
def test_couette_with_floating_subdomains_and_stokes_stokes_mortars(element):
    """4 x 2 Stokes subdomains (two floating, FETI) over 8 x 4 Darcy: the
    Stokes-Stokes mortars carry the constant shear stress vector.  The
    Couette field lies in both the rectangular and the triangular spaces."""
    p = _couette("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})
    p["discretization"] = {"stokes": element}
    o = Oracle(p)
    assert o.G.shape[1] == 4
    for l in (0, 3000):
        f, it, rel, ok = o.realization_S3(l, rtol=1e-13)
        assert ok
        assert _couette_error(o, f) < 1e-9


@pytest.mark.parametrize("mistake", ["alpha_over_K", "dropped_h"])
def test_couette_pin_catches_planted_bjs_mistakes(monkeypatch, mistake):
    if mistake == "alpha_over_K":
        monkeypatch.setattr(ostokes, "bjs_coefficient", lambda nu, a, k: nu * a / k)
    else:
        orig = ostokes.bjs_edge_mass
        monkeypatch.setattr(ostokes, "bjs_edge_mass", lambda coef, h: orig(coef, 1.0))
    o = Oracle(_couette("cfg0"))
    f, it, rel, ok = o.realization_S3(5, rtol=1e-13)
    assert ok
    assert _couette_error(o, f) > 1e-3


# ---------------------------------------------------------------------------
# small non-matching layout with P2 mortars
# ---------------------------------------------------------------------------
def _nonmatching(sigma2=1.0, elements=2):
    """Stokes [0,1]x[1,2] as 2 subdomains over Darcy [0,1]x[0,1] as 2x2
    subdomains with pairwise different meshes (every Darcy-Darcy and
    Stokes-Darcy interface is non-matching); P2 mortars; two KL regions
    (left and right Darcy columns)."""
    stokes = [{"type": "stokes", "rect": [0.0, 0.5, 1.0, 2.0], "n": [6, 8], "region": -1},
              {"type": "stokes", "rect": [0.5, 1.0, 1.0, 2.0], "n": [8, 6], "region": -1}]
    meshes = [(6, 8), (10, 6), (8, 10), (6, 6)]
    darcy = []
    for k, (jx, jy) in enumerate([(0, 0), (1, 0), (0, 1), (1, 1)]):
        darcy.append({"type": "darcy", "rect": [0.5 * jx, 0.5 * jx + 0.5, 0.5 * jy, 0.5 * jy + 0.5],
                      "n": list(meshes[k]), "region": jx})
    regions = [{"rect": [0.5 * r, 0.5 * r + 0.5, 0.0, 1.0], "nterm": 2, "sigma2": sigma2, "eta": [0.3, 0.2],
                "mean_logk": 0.0} for r in range(2)]
    return {"name": "nonmatching", "domain": [0.0, 1.0, 0.0, 2.0],
            "physics": {"nu_s": 1.0, "nu_d": 1.0, "alpha": 1.0, "k_bjs": 1.0, "inflow": [0.0, -1.0],
                        "p_bottom": 0.0},
            "subdomains": stokes + darcy, "mortar": {"degree": 2, "elements": elements},
            "regions": regions, "rule": {"kind": "tensor", "m": 2}}


def _lagrange(nodes, k):
    """k-th Lagrange polynomial through `nodes` (written out, independent of
    the oracle's shape functions)."""
    others = [x for j, x in enumerate(nodes) if j != k]

    def f(t):
        v = 1.0
        for x in others:
            v *= (t - x) / (nodes[k] - x)
        return v
    return f


def _mortar_fn(fa, q):
    """The scalar mortar basis function of scalar node q of interface fa."""
    e, a = divmod(q, fa.deg + 1)
    t0 = fa.a + e * fa.H
    nodes = [t0 + fa.H * s for s in np.linspace(0.0, 1.0, fa.deg + 1)]
    lag = _lagrange(nodes, a)
    return (lambda t: lag(t) if t0 - 1e-14 <= t <= t0 + fa.H + 1e-14 else 0.0), t0, t0 + fa.H


def _side_of(L, i, fa):
    x0, x1, y0, y1 = L.subs[i]["rect"]
    if fa.orient == "h":
        return ("bottom", (0.0, -1.0)) if abs(fa.coord - y0) < 1e-12 else ("top", (0.0, 1.0))
    return ("left", (-1.0, 0.0)) if abs(fa.coord - x0) < 1e-12 else ("right", (1.0, 0.0))


def _vel(x, y):
    """A velocity field quadratic in each variable (exact in Q2)."""
    return np.array([x * x - 0.3 * x * y + 0.2, y * y + 0.5 * x - 0.1 * x * y - 0.1])


@pytest.mark.parametrize("elements", [1, 2])
def test_stokes_mortar_coupling_against_quadrature(elements):
    L = Layout(_nonmatching(elements=elements))
    for i in (0, 1):
        st = StokesLocal(L, i)
        x0, x1, y0, y1 = L.subs[i]["rect"]
        X = x0 + 0.5 * st.hx * np.arange(st.nnx)
        Y = y0 + 0.5 * st.hy * np.arange(st.nny)
        XX, YY = np.meshgrid(X, Y)
        v = _vel(XX.ravel(), YY.ravel())
        vn = np.empty(st.nvel)
        vn[0::2], vn[1::2] = v[0], v[1]
        got = st.Q @ vn
        for fi in L.sub_ifaces[i]:
            fa = L.ifaces[fi]
            side, nrm = _side_of(L, i, fa)
            cut = [fa.a + e * fa.H for e in range(fa.nelem + 1)]
            h = st.hx if fa.orient == "h" else st.hy
            fine = list(np.arange(fa.a, fa.b + 1e-12, h))
            for q in range(fa.nnode):
                mu, ta, tb = _mortar_fn(fa, q)
                pts = sorted(set([t for t in cut + fine if ta - 1e-12 <= t <= tb + 1e-12]))

                def trace(t, c):
                    xy = (t, fa.coord) if fa.orient == "h" else (fa.coord, t)
                    return _vel(*xy)[c]
                if fa.kind == "ss":
                    for c in range(2):
                        want = quad(lambda t: mu(t) * trace(t, c), ta, tb, points=pts[1:-1], epsabs=1e-14,
                                    epsrel=1e-13)[0]
                        loc = L.local_index(i, fa, 2 * q + c)
                        assert abs(got[loc] - L.sub_sign[i][loc] * want) < 1e-12
                else:
                    want = quad(lambda t: mu(t) * (nrm[0] * trace(t, 0) + nrm[1] * trace(t, 1)), ta, tb,
                                points=pts[1:-1], epsabs=1e-14, epsrel=1e-13)[0]
                    assert abs(got[L.local_index(i, fa, q)] - want) < 1e-12


def test_darcy_edge_averages_against_quadrature():
    from oracle.darcy import DarcyLocal
    L = Layout(_nonmatching())
    for i in range(2, 6):
        dl = DarcyLocal(L, i, np.ones(L.subs[i]["n"][0] * L.subs[i]["n"][1]))
        for k, be in enumerate(dl.medges):
            fa = L.ifaces[be["iface"]]
            for q in range(fa.nnode):
                mu, ta, tb = _mortar_fn(fa, q)
                lo, hi = max(ta, be["t0"]), min(tb, be["t1"])
                want = 0.0
                if hi > lo:
                    want = quad(mu, lo, hi, epsabs=1e-15, epsrel=1e-13)[0] / be["length"]
                assert abs(dl.avg[k, L.local_index(i, fa, q)] - want) < 1e-13


def _nonmatching_closed_form_error(o):
    """Deviation from u = (0, -1), p_d = y, p_s = 1, lambda = trace of p."""
    f, it, rel, ok = o.realization_S2(0, rtol=1e-13)
    assert ok
    L = o.L
    err = max(np.abs(f["stokes_u"][0::2]).max(), np.abs(f["stokes_u"][1::2] + 1.0).max(),
              np.abs(f["stokes_p"] - 1.0).max())
    off = 0
    for i in o.darcy_ids:
        nx, ny = L.subs[i]["n"]
        y0, y1 = L.subs[i]["rect"][2:]
        yc = y0 + (np.arange(ny) + 0.5) * (y1 - y0) / ny
        err = max(err, np.abs(f["darcy_p"][off:off + nx * ny].reshape(ny, nx) - yc[:, None]).max())
        off += nx * ny
    lam = f["lambda"]
    for fa in L.ifaces:
        v = lam[fa.off:fa.off + fa.ndof]
        t = np.array([fa.a + (e + s) * fa.H for e in range(fa.nelem) for s in np.linspace(0, 1, fa.deg + 1)])
        if fa.kind == "ss":
            want = np.tile([1.0, 0.0] if fa.orient == "v" else [0.0, 1.0], t.size)
        elif fa.kind == "sd":
            want = np.ones(t.size)
        else:
            want = t if fa.orient == "v" else np.full(t.size, fa.coord)
        err = max(err, np.abs(v - want).max())
    return err


def test_closed_form_on_nonmatching_p2_layout():
    o = Oracle(_nonmatching(sigma2=0.0))
    assert _nonmatching_closed_form_error(o) < 1e-10


def test_closed_form_on_small_cfg3_layout():
    """The cfg3 geometry (8 Stokes, 32 Darcy, P2 mortar, 8 KL regions) with
    small non-matching Darcy meshes and sigma^2 = 0."""
    p = problem("cfg3", sigma2=0.0, stokes_mesh=(8, 8))
    rng = np.random.default_rng(11)
    for s in p["subdomains"]:
        if s["type"] == "darcy":
            s["n"] = [int(rng.choice([8, 10, 12])), int(rng.choice([8, 10, 12]))]
    p["mortar"] = {"degree": 2, "elements": 2}
    p["rule"] = {"kind": "sparse", "level": 1, "growth": "paper"}
    o = Oracle(p)
    assert _nonmatching_closed_form_error(o) < 1e-10


def test_p2_closed_form_catches_swapped_p2_nodes(monkeypatch):
    orig = geom.mortar_shape

    def swapped(deg, s):
        v = orig(deg, s)
        return v[[0, 2, 1]] if deg == 2 else v
    monkeypatch.setattr(geom, "mortar_shape", swapped)
    o = Oracle(_nonmatching(sigma2=0.0))
    assert _nonmatching_closed_form_error(o) > 1e-3


@pytest.mark.parametrize("l", [3, 12])
def test_all_methods_match_monolithic_on_nonmatching_p2_layout(l):
    o = Oracle(_nonmatching(sigma2=1.0))
    y = o.grid.points[l]
    Kd = {i: o.darcy_K(i, o.region_point(y, o.L.subs[i]["region"])) for i in o.darcy_ids}
    m = monolithic.solve(o.L, Kd, o.stokes)
    for meth in ("S1", "S2", "S3"):
        f, it, rel, ok = getattr(o, "realization_" + meth)(l, rtol=1e-12)
        assert ok
        for k in FIELDS:
            assert np.abs(f[k] - m[k]).max() <= 1e-9 * max(np.abs(m[k]).max(), 1e-300), (meth, k)
