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
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


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
        # mortar edge averages: avg[e_local, q_local] for mortar boundary edges
        R = layout.sub_dofs[i].size
        self.R = R
        self.medges = [be for be in self.bedges if be["kind"] == "mortar"]
        self.avg = np.zeros((len(self.medges), R))
        for k, be in enumerate(self.medges):
            f = layout.ifaces[be["iface"]]
            ints = f.node_integrals(be["t0"], be["t1"])
            base = layout.local_index(i, f, 0)
            self.avg[k, base: base + f.ndof] = ints / be["length"]

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
