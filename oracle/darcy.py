"""Darcy subdomain problems with RT0-Q0 (oracle).

Section 5.1, eqs. (starDproblem1-2) and (barDproblem1-2): on a Darcy
subdomain the interface datum is a pressure lambda; the local problem is
nu_d K^{-1} u + grad p = 0, div u = 0 with p = lambda on Gamma_i, the outer
data on the rest of the boundary, and the interface operator reads back the
normal flux tested with the mortar functions (eq. interface).

Reading: the RT0 velocity mass matrix is integrated with the trapezoidal
(vertex) rule, which makes it diagonal; eliminating the edge velocities
leaves the 5-point cell-centred system with harmonic transmissibilities
  interior edge:  T = |e| / (nu_d (h/2)(1/K_L + 1/K_R)),  U = T (p_L - p_R)
  Dirichlet edge: T = 2 |e| K_c / (nu_d h),               U_out = T (p_c - avg_e g)
  no-flow edge:   U = 0
where h is the cell size normal to the edge and U the edge flux.

The alternative is the exactly integrated RT0 mass (the discretization of
the paper's numerical cases, Section 6), solved in hybridized form: on a
cell of size hx x hy with permeability K the normal-velocity basis of the
two x-faces (and likewise the two y-faces) gives the mass
  nu |c| / K [[1/3, 1/6], [1/6, 1/3]]
in +x / +y oriented velocities.  With outward face fluxes U, cell pressure
p and face pressures mu the cell equations are  M U - p 1 + mu = 0  and
1^T U = 0, so  U = M^{-1} (p 1 - mu),  p = (1^T M^{-1} mu) / (1^T M^{-1} 1)
and  U = -H mu  with  H = M^{-1} - M^{-1} 1 1^T M^{-1} / (1^T M^{-1} 1).
Flux continuity on interior edges and U = 0 on no-flow edges give an SPD
system for the unknown face pressures; mortar edges carry mu = the edge
average of lambda, outer Dirichlet edges the outer pressure.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def darcy_mass(layout):
    """'trapezoidal' (diagonal mass, cell-centred system) or 'exact'."""
    m = layout.prob.get("discretization", {}).get("darcy", "trapezoidal")
    if m not in ("trapezoidal", "exact"):
        raise ValueError("unknown Darcy mass %r" % m)
    return m


def make_darcy_local(layout, i, K):
    """The local Darcy solver of the problem's discretization."""
    if darcy_mass(layout) == "exact":
        return DarcyLocalExact(layout, i, K)
    return DarcyLocal(layout, i, K)


def _mortar_averages(layout, i, bedges):
    """R, the mortar edges, and avg[e_local, q_local]: the average over each
    mortar edge of every local mortar basis function."""
    R = layout.sub_dofs[i].size
    medges = [be for be in bedges if be["kind"] == "mortar"]
    avg = np.zeros((len(medges), R))
    for k, be in enumerate(medges):
        f = layout.ifaces[be["iface"]]
        ints = f.node_integrals(be["t0"], be["t1"])
        base = layout.local_index(i, f, 0)
        avg[k, base: base + f.ndof] = ints / be["length"]
    return R, medges, avg


class DarcyLocal:
    """Local CCFD operator of one Darcy subdomain for one permeability field."""

    def __init__(self, layout, i, K):
        self.layout, self.i = layout, i
        s = layout.subs[i]
        self.nx, self.ny = s["n"]
        self.hx, self.hy = s["h"]
        nu = float(layout.phys["nu_d"])
        self.nu = nu
        self.K = np.asarray(K, dtype=np.float64)
        nx, ny, hx, hy = self.nx, self.ny, self.hx, self.hy
        N = nx * ny
        self.N = N
        rows, cols, vals = [], [], []
        diag = np.zeros(N)
        # interior vertical edges
        self.int_edges = []  # (edge index, cell L, cell R, T)
        for iy in range(ny):
            for ix in range(1, nx):
                cL, cR = iy * nx + ix - 1, iy * nx + ix
                T = hy / (nu * (hx / 2.0) * (1.0 / K[cL] + 1.0 / K[cR]))
                self.int_edges.append((iy * (nx + 1) + ix, cL, cR, T))
        nv = (nx + 1) * ny
        for iy in range(1, ny):
            for ix in range(nx):
                cB, cT = (iy - 1) * nx + ix, iy * nx + ix
                T = hx / (nu * (hy / 2.0) * (1.0 / K[cB] + 1.0 / K[cT]))
                self.int_edges.append((nv + iy * nx + ix, cB, cT, T))
        for _, a, b, T in self.int_edges:
            diag[a] += T
            diag[b] += T
            rows += [a, b]
            cols += [b, a]
            vals += [-T, -T]
        # boundary edges
        self.bedges = layout.darcy_boundary(i)
        for be in self.bedges:
            if be["kind"] == "noflow":
                be["T"] = 0.0
                continue
            be["T"] = 2.0 * be["length"] * K[be["cell"]] / (nu * be["hperp"])
            diag[be["cell"]] += be["T"]
        rows += list(range(N))
        cols += list(range(N))
        vals += diag.tolist()
        self.P = sp.csc_matrix((vals, (rows, cols)), shape=(N, N))
        self._lu = None
        self.R, self.medges, self.avg = _mortar_averages(layout, i, self.bedges)

    def lu(self):
        if self._lu is None:
            self._lu = spla.splu(self.P)
        return self._lu

    def solve(self, lam_local, p_outer=0.0):
        """Pressure and boundary fluxes for interface pressure lam_local (local mortar coeffs).

        p_outer is the outer Dirichlet pressure (the complementary problem
        carries it; the interface problem has it zero).
        """
        lamb = self.avg @ np.asarray(lam_local, dtype=np.float64)
        rhs = np.zeros(self.N)
        for k, be in enumerate(self.medges):
            rhs[be["cell"]] += be["T"] * lamb[k]
        for be in self.bedges:
            if be["kind"] == "dirichlet":
                rhs[be["cell"]] += be["T"] * p_outer
        p = self.lu().solve(rhs)
        uout = np.array([be["T"] * (p[be["cell"]] - lamb[k]) for k, be in enumerate(self.medges)])
        return p, uout

    def response(self, lam_local):
        """S_{H,i} lambda: minus the outward flux tested with every mortar function."""
        _, uout = self.solve(lam_local)
        return -(self.avg.T @ uout)

    def basis(self):
        """Multiscale flux basis: the columns S_{H,i} xi^j, one local solve per mortar DOF."""
        S = np.zeros((self.R, self.R))
        for j in range(self.R):
            e = np.zeros(self.R)
            e[j] = 1.0
            S[:, j] = self.response(e)
        return S

    def velocities(self, p, lam_local, p_outer=0.0):
        """RT0 normal velocities u_e = flux / |e| on all edges (+x / +y orientation)."""
        nx, ny = self.nx, self.ny
        ne = (nx + 1) * ny + nx * (ny + 1)
        u = np.zeros(ne)
        for e, a, b, T in self.int_edges:
            ln = self.hy if e < (nx + 1) * ny else self.hx
            u[e] = T * (p[a] - p[b]) / ln
        lamb = self.avg @ np.asarray(lam_local, dtype=np.float64)
        k = 0
        for be in self.bedges:
            if be["kind"] == "mortar":
                uo = be["T"] * (p[be["cell"]] - lamb[k])
                k += 1
            elif be["kind"] == "dirichlet":
                uo = be["T"] * (p[be["cell"]] - p_outer)
            else:
                uo = 0.0
            u[be["edge"]] = be["sgn"] * uo / be["length"]
        return u


class DarcyLocalExact:
    """Hybridized RT0-Q0 of one Darcy subdomain with the exact velocity mass.

    Edges are numbered as in DarcyLocal.velocities: the (nx + 1) ny vertical
    edges row by row, then the nx (ny + 1) horizontal ones.  The unknowns are
    the face pressures mu of the interior and no-flow edges."""

    def __init__(self, layout, i, K):
        self.layout, self.i = layout, i
        s = layout.subs[i]
        self.nx, self.ny = s["n"]
        self.hx, self.hy = s["h"]
        nu = float(layout.phys["nu_d"])
        self.nu = nu
        self.K = np.asarray(K, dtype=np.float64)
        nx, ny, hx, hy = self.nx, self.ny, self.hx, self.hy
        self.N = nx * ny
        nv = (nx + 1) * ny
        self.nv = nv
        self.ne = nv + nx * (ny + 1)
        # faces of every cell in the order (left, right, bottom, top)
        self.faces = np.array([[iy * (nx + 1) + ix, iy * (nx + 1) + ix + 1, nv + iy * nx + ix,
                                nv + (iy + 1) * nx + ix] for iy in range(ny) for ix in range(nx)])
        # outward flux U of a face -> +x / +y velocity: -U/|e| on left/bottom faces
        self.face_sign = np.array([-1.0, 1.0, -1.0, 1.0])
        self.face_len = np.array([hy, hy, hx, hx])
        self.Minv, self.H, self.w = [], [], []
        rows, cols, vals = [], [], []
        one = np.ones(4)
        for c in range(self.N):
            Mc = self.cell_mass_fluxes(c)
            Mi = np.linalg.inv(Mc)
            m1 = Mi @ one
            sc = one @ m1
            H = Mi - np.outer(m1, m1) / sc
            self.Minv.append(Mi)
            self.H.append(H)
            self.w.append(m1 / sc)
            f = self.faces[c]
            r, cc = np.meshgrid(f, f, indexing="ij")
            rows.append(r.ravel())
            cols.append(cc.ravel())
            vals.append(H.ravel())
        self.Hg = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(self.ne, self.ne)).tocsr()
        self.bedges = layout.darcy_boundary(i)
        known = np.zeros(self.ne, dtype=bool)
        for be in self.bedges:
            if be["kind"] in ("mortar", "dirichlet"):
                known[be["edge"]] = True
        self.known = np.nonzero(known)[0]
        self.unknown = np.nonzero(~known)[0]
        self.Huu = self.Hg[self.unknown][:, self.unknown].tocsc()
        self.Huk = self.Hg[self.unknown][:, self.known]
        self._lu = None
        self.R, self.medges, self.avg = _mortar_averages(layout, i, self.bedges)

    def cell_mass_fluxes(self, c):
        """Exact RT0 mass of cell c in outward face fluxes (left, right, bottom, top).

        In +x / +y velocities a face pair has nu |c| / K [[1/3, 1/6], [1/6, 1/3]];
        a flux is the velocity times the face length, outward on right/top."""
        nu, hx, hy, K = self.nu, self.hx, self.hy, self.K[c]
        pair = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]]) * nu * hx * hy / K
        M = np.zeros((4, 4))
        S = np.diag(self.face_sign / self.face_len)   # outward flux -> oriented velocity
        M[:2, :2] = pair
        M[2:, 2:] = pair
        return S @ M @ S

    def lu(self):
        if self._lu is None:
            self._lu = spla.splu(self.Huu)
        return self._lu

    def face_pressures(self, lam_local, p_outer=0.0):
        mu = np.zeros(self.ne)
        lamb = self.avg @ np.asarray(lam_local, dtype=np.float64)
        for k, be in enumerate(self.medges):
            mu[be["edge"]] = lamb[k]
        for be in self.bedges:
            if be["kind"] == "dirichlet":
                mu[be["edge"]] = p_outer
        mu[self.unknown] = self.lu().solve(-(self.Huk @ mu[self.known]))
        return mu

    def cell_fluxes(self, mu):
        """Cell pressures and the outward face fluxes of every cell."""
        p = np.array([self.w[c] @ mu[self.faces[c]] for c in range(self.N)])
        U = np.array([self.Minv[c] @ (p[c] - mu[self.faces[c]]) for c in range(self.N)])
        return p, U

    def _boundary_flux(self, be, U):
        c = be["cell"]
        k = list(self.faces[c]).index(be["edge"])
        return U[c, k]

    def solve(self, lam_local, p_outer=0.0):
        """Cell pressures and outward mortar-edge fluxes (as DarcyLocal.solve)."""
        mu = self.face_pressures(lam_local, p_outer)
        p, U = self.cell_fluxes(mu)
        uout = np.array([self._boundary_flux(be, U) for be in self.medges])
        return p, uout

    def response(self, lam_local):
        _, uout = self.solve(lam_local)
        return -(self.avg.T @ uout)

    def basis(self):
        S = np.zeros((self.R, self.R))
        for j in range(self.R):
            e = np.zeros(self.R)
            e[j] = 1.0
            S[:, j] = self.response(e)
        return S

    def velocities(self, p, lam_local, p_outer=0.0):
        """RT0 normal velocities on all edges (+x / +y orientation)."""
        mu = self.face_pressures(lam_local, p_outer)
        _, U = self.cell_fluxes(mu)
        u = np.zeros(self.ne)
        # every edge from one of its cells (interior edges agree to rounding)
        for c in range(self.N):
            for k in range(4):
                u[self.faces[c][k]] = self.face_sign[k] * U[c, k] / self.face_len[k]
        return u
