"""Subdomains, interfaces, mortar spaces and index maps (oracle).

Follows Section 3.1 (domain decomposition: Stokes subdomains first, then
Darcy; interfaces Gamma_ss, Gamma_sd, Gamma_dd between adjacent subdomains)
and Section 3.3 (a coarse mortar space on every interface; scalar on
Gamma_sd and Gamma_dd, a 2-vector on Gamma_ss).  Orderings are not fixed by
the paper; this module takes the following reading:

* interfaces are the subdomain pairs (i < j) whose boundaries share a
  segment of positive length, ordered by (i, j);
* the mortar on an interface is discontinuous Lagrange of degree 1 or 2 on
  E uniform elements along x (horizontal interface) or y (vertical one);
  DOF order inside an interface is (element, node, component);
* subdomain i sees the mortar DOFs of its interfaces in interface order; on
  a Stokes-Stokes interface the jump [v] = v_i - v_j of the coupling form
  b_Lambda gives the lower-numbered subdomain the sign +1 and the other -1;
* Darcy cells are row-major (x fastest); RT0 edges are the vertical edges
  row-major, then the horizontal edges row-major; Q2 velocity nodes and Q1
  pressure nodes are row-major.
"""
import numpy as np

GL3_X = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
GL3_W = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])
TOL = 1e-12


def mortar_shape(deg, s):
    """Lagrange shape values on [0, 1]; P1 nodes {0, 1}, P2 nodes {0, 1/2, 1}."""
    s = np.asarray(s, dtype=np.float64)
    if deg == 1:
        return np.stack([1.0 - s, s])
    if deg == 2:
        return np.stack([2.0 * (s - 0.5) * (s - 1.0), -4.0 * s * (s - 1.0), 2.0 * s * (s - 0.5)])
    raise ValueError("mortar degree must be 1 or 2")


class Interface:
    def __init__(self, idx, i, j, kind, orient, coord, a, b, ncomp, nelem, deg, off):
        self.idx, self.i, self.j, self.kind = idx, i, j, kind
        self.orient, self.coord, self.a, self.b = orient, coord, a, b
        self.ncomp, self.nelem, self.deg, self.off = ncomp, nelem, deg, off
        self.nnode = nelem * (deg + 1)
        self.ndof = self.nnode * ncomp
        self.H = (b - a) / nelem

    def node_integrals(self, t0, t1, g=None):
        """Integrals over [t0, t1] of every scalar mortar node shape times g(t).

        Exact integration over the common refinement of [t0, t1] and the
        mortar mesh with 3-point Gauss-Legendre per piece (exact to degree
        five, enough for a quadratic mortar times a quadratic trace).
        """
        cuts = [t0]
        for e in range(1, self.nelem):
            x = self.a + e * self.H
            if t0 + TOL < x < t1 - TOL:
                cuts.append(x)
        cuts.append(t1)
        out = np.zeros(self.nnode)
        for p0, p1 in zip(cuts[:-1], cuts[1:]):
            half = 0.5 * (p1 - p0)
            mid = 0.5 * (p1 + p0)
            tq = mid + half * GL3_X
            wq = half * GL3_W
            e = int(np.floor((0.5 * (p0 + p1) - self.a) / self.H))
            e = min(max(e, 0), self.nelem - 1)
            s = (tq - (self.a + e * self.H)) / self.H
            shp = mortar_shape(self.deg, s)
            gv = np.ones_like(tq) if g is None else g(tq)
            out[e * (self.deg + 1): (e + 1) * (self.deg + 1)] += shp @ (wq * gv)
        return out

    def eval_nodes(self, t):
        """Values of all scalar mortar node shapes at points t (nnode x len(t))."""
        t = np.atleast_1d(np.asarray(t, dtype=np.float64))
        out = np.zeros((self.nnode, t.size))
        e = np.clip(np.floor((t - self.a) / self.H).astype(int), 0, self.nelem - 1)
        s = (t - (self.a + e * self.H)) / self.H
        shp = mortar_shape(self.deg, s)
        for q in range(t.size):
            out[e[q] * (self.deg + 1):(e[q] + 1) * (self.deg + 1), q] = shp[:, q]
        return out


class Layout:
    """Geometry and index maps of one problem (Section 3.1, 3.3)."""

    def __init__(self, prob):
        self.prob = prob
        self.phys = prob["physics"]
        self.domain = prob["domain"]
        self.subs = []
        for s in prob["subdomains"]:
            x0, x1, y0, y1 = [float(v) for v in s["rect"]]
            nx, ny = int(s["n"][0]), int(s["n"][1])
            self.subs.append({"type": s["type"], "rect": (x0, x1, y0, y1), "n": (nx, ny),
                              "h": ((x1 - x0) / nx, (y1 - y0) / ny), "region": int(s["region"])})
        self.nsub = len(self.subs)
        types = [s["type"] for s in self.subs]
        self.n_stokes = types.count("stokes")
        if types != ["stokes"] * self.n_stokes + ["darcy"] * (self.nsub - self.n_stokes):
            raise ValueError("Stokes subdomains must be numbered before Darcy subdomains")
        deg = int(prob["mortar"]["degree"])
        nel = int(prob["mortar"]["elements"])
        self.ifaces = []
        off = 0
        for i in range(self.nsub):
            for j in range(i + 1, self.nsub):
                seg = _shared(self.subs[i]["rect"], self.subs[j]["rect"])
                if seg is None:
                    continue
                orient, coord, a, b = seg
                ti, tj = types[i], types[j]
                kind = "ss" if ti == tj == "stokes" else ("dd" if ti == tj == "darcy" else "sd")
                ncomp = 2 if kind == "ss" else 1
                f = Interface(len(self.ifaces), i, j, kind, orient, coord, a, b, ncomp, nel, deg, off)
                off += f.ndof
                self.ifaces.append(f)
        self.M = off
        # per-subdomain mortar DOF lists (global index, sign)
        self.sub_ifaces = [[] for _ in range(self.nsub)]
        for f in self.ifaces:
            self.sub_ifaces[f.i].append(f.idx)
            self.sub_ifaces[f.j].append(f.idx)
        self.sub_dofs, self.sub_sign, self.sub_dof_off = [], [], []
        for i in range(self.nsub):
            g, sg, offs = [], [], {}
            for fi in self.sub_ifaces[i]:
                f = self.ifaces[fi]
                offs[fi] = len(g)
                sign = -1.0 if (f.kind == "ss" and f.j == i) else 1.0
                g.extend(range(f.off, f.off + f.ndof))
                sg.extend([sign] * f.ndof)
            self.sub_dofs.append(np.array(g, dtype=np.int64))
            self.sub_sign.append(np.array(sg))
            self.sub_dof_off.append(offs)
        # KL regions
        self.regions = prob["regions"]
        for i, s in enumerate(self.subs):
            if s["type"] == "darcy":
                r = self.regions[s["region"]]["rect"]
                x0, x1, y0, y1 = s["rect"]
                if not (x0 >= r[0] - TOL and x1 <= r[1] + TOL and y0 >= r[2] - TOL and y1 <= r[3] + TOL):
                    raise ValueError("a Darcy subdomain must lie inside its KL region")

    # ---- side classification -------------------------------------------------
    def side_segment(self, i, side):
        x0, x1, y0, y1 = self.subs[i]["rect"]
        return {"left": ("v", x0, y0, y1), "right": ("v", x1, y0, y1),
                "bottom": ("h", y0, x0, x1), "top": ("h", y1, x0, x1)}[side]

    def iface_at(self, i, side, t):
        """Interface of subdomain i containing the point at tangential coord t on a side."""
        orient, c, a, b = self.side_segment(i, side)
        for fi in self.sub_ifaces[i]:
            f = self.ifaces[fi]
            if f.orient == orient and abs(f.coord - c) < TOL and f.a - TOL <= t <= f.b + TOL:
                return f
        return None

    def side_is_outer(self, i, side):
        orient, c, a, b = self.side_segment(i, side)
        mid = 0.5 * (a + b)
        return self.iface_at(i, side, mid) is None

    def is_floating(self, i):
        """A Stokes subdomain without any outer (Dirichlet) side is floating."""
        return self.subs[i]["type"] == "stokes" and not any(
            self.side_is_outer(i, s) for s in ("left", "right", "bottom", "top"))

    # ---- Darcy index maps ----------------------------------------------------
    def darcy_edges(self, i):
        """Per RT0 edge: (orientation, ix, iy) following the edge numbering."""
        nx, ny = self.subs[i]["n"]
        out = [("v", ix, iy) for iy in range(ny) for ix in range(nx + 1)]
        out += [("h", ix, iy) for iy in range(ny + 1) for ix in range(nx)]
        return out

    def darcy_boundary(self, i):
        """Boundary edges of Darcy subdomain i.

        Returns a list of dicts (edge, cell, side, kind, iface, t0, t1, length,
        hperp, sgn) where kind is "mortar", "dirichlet" (outer p data) or
        "noflow", and sgn = +1 when the outward normal is +x / +y.
        """
        s = self.subs[i]
        nx, ny = s["n"]
        hx, hy = s["h"]
        x0, x1, y0, y1 = s["rect"]
        nv = (nx + 1) * ny
        out = []
        for side in ("bottom", "top", "left", "right"):
            if side in ("bottom", "top"):
                iy = 0 if side == "bottom" else ny
                cy = 0 if side == "bottom" else ny - 1
                for ix in range(nx):
                    t0, t1 = x0 + ix * hx, x0 + (ix + 1) * hx
                    out.append(self._bedge(i, side, nv + iy * nx + ix, cy * nx + ix, t0, t1, hx, hy,
                                           -1.0 if side == "bottom" else 1.0))
            else:
                ix = 0 if side == "left" else nx
                cx = 0 if side == "left" else nx - 1
                for iy in range(ny):
                    t0, t1 = y0 + iy * hy, y0 + (iy + 1) * hy
                    out.append(self._bedge(i, side, iy * (nx + 1) + ix, iy * nx + cx, t0, t1, hy, hx,
                                           -1.0 if side == "left" else 1.0))
        return out

    def _bedge(self, i, side, edge, cell, t0, t1, length, hperp, sgn):
        f = self.iface_at(i, side, 0.5 * (t0 + t1))
        if f is not None:
            kind = "mortar"
        else:
            ymin = self.domain[2]
            orient, c, a, b = self.side_segment(i, side)
            kind = "dirichlet" if (side == "bottom" and abs(c - ymin) < TOL) else "noflow"
        return {"edge": edge, "cell": cell, "side": side, "kind": kind,
                "iface": None if f is None else f.idx, "t0": t0, "t1": t1,
                "length": length, "hperp": hperp, "sgn": sgn}

    def local_index(self, i, f, q):
        """Position of DOF q of interface f in subdomain i's local mortar list."""
        return self.sub_dof_off[i][f.idx] + q


def _shared(r1, r2):
    ax0, ax1, ay0, ay1 = r1
    bx0, bx1, by0, by1 = r2
    for c1, c2 in ((ay1, by0), (ay0, by1)):
        if abs(c1 - c2) < TOL:
            a, b = max(ax0, bx0), min(ax1, bx1)
            if b - a > TOL:
                return ("h", c1, a, b)
    for c1, c2 in ((ax1, bx0), (ax0, bx1)):
        if abs(c1 - c2) < TOL:
            a, b = max(ay0, by0), min(ay1, by1)
            if b - a > TOL:
                return ("v", c1, a, b)
    return None


def index_maps(layout):
    """Integer maps compared bit-exactly against the library.

    interfaces : (n_if, 5) rows (i, j, kind 0=ss 1=sd 2=dd, ndof, offset)
    sub_dofs   : concatenated per-subdomain global mortar DOFs
    sub_ptr    : CSR pointer into sub_dofs
    sub_sign   : concatenated signs (+1 / -1)
    """
    kinds = {"ss": 0, "sd": 1, "dd": 2}
    ifs = np.array([[f.i, f.j, kinds[f.kind], f.ndof, f.off] for f in layout.ifaces], dtype=np.int64)
    ptr = np.zeros(layout.nsub + 1, dtype=np.int64)
    for i in range(layout.nsub):
        ptr[i + 1] = ptr[i] + layout.sub_dofs[i].size
    return {"interfaces": ifs, "sub_dofs": np.concatenate(layout.sub_dofs), "sub_ptr": ptr,
            "sub_sign": np.concatenate(layout.sub_sign).astype(np.int64)}
