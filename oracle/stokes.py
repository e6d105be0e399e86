"""Stokes subdomain problems with Taylor-Hood Q2-Q1 on rectangles (oracle).

Section 3.2 (forms a~_i with the BJS term on Gamma_i n Gamma_sd, b~_i) and
Section 5.1, eqs. (starSproblem1-2) and (barSproblem1-2): the interface
datum is a normal stress (a stress vector on Gamma_ss); the local problem is
a Neumann problem, and its velocity trace tested with the mortar functions
gives the interface operator.  Floating subdomains (no outer boundary) are
solved in V / ker a~_i as FETI does (Section 1, Section 5.1): the load is
projected onto the compatible loads and the solution is taken orthogonal
(in the Euclidean coefficient inner product) to the kernel Z_i of rigid
motions that the BJS term leaves free.

Readings: Q2-Q1 on rectangles by default; 3x3 Gauss per element.  The
triangular Taylor-Hood pair P2-P1 of the paper's numerical cases (Section 6)
is the alternative element: every rectangle is cut into two right triangles
along a diagonal, which puts the P2 nodes on the same (2nx+1) x (2ny+1) node
grid as Q2 (the diagonal midpoint is the rectangle centre) and the P1
pressures on the Q1 vertices, so both pairs share every index map.  The
diagonal runs from the lower-left to the upper-right corner except in the
lower-right and upper-left corner rectangles of a subdomain, which take the
other diagonal, so that no triangle has two edges on the subdomain boundary.
P2-P1 integrals use the edge-midpoint rule, exact for the degree-2
integrands of both forms.  The velocity (inflow, optionally
with a linear shear profile in y) is imposed on the whole Stokes outer
boundary; the BJS coefficient uses the deterministic
permeability k_bjs, so every Stokes operator is deterministic.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .geometry import GL3_W, GL3_X

_Q = 0.5 * (1.0 + GL3_X)
_W = 0.5 * GL3_W


def _l2(s):
    return np.stack([2 * (s - 0.5) * (s - 1), -4 * s * (s - 1), 2 * s * (s - 0.5)])


def _dl2(s):
    return np.stack([4 * s - 3, -8 * s + 4, 4 * s - 1])


def _l1(s):
    return np.stack([1 - s, s])


def bjs_coefficient(nu, alpha, k_bjs):
    """Friction coefficient of the BJS condition (Section 2, eq. BJS):
    nu alpha / sqrt(K) with the deterministic permeability of the BJS term."""
    return nu * alpha / np.sqrt(k_bjs)


def bjs_edge_mass(coef, h):
    """3x3 matrix of coef * int u_tau v_tau over one fine edge of length h for
    the three Q2 trace nodes of that edge (the BJS term of the form a~_i of
    Section 3.2), by 3-point Gauss on [0, 1] scaled by h."""
    m = np.zeros((3, 3))
    for qk, sq in enumerate(_Q):
        Lv = _l2(sq)
        m += _W[qk] * np.outer(Lv, Lv)
    return coef * h * m


def element_matrices(hx, hy, nu):
    """18x18 velocity block (DOF 2*node+comp, node = 3*b+a) and 4x18 divergence block."""
    A = np.zeros((18, 18))
    B = np.zeros((4, 18))
    for qi, s in enumerate(_Q):
        for qj, t in enumerate(_Q):
            w = _W[qi] * _W[qj] * hx * hy
            Ls, Lt, dLs, dLt = _l2(s), _l2(t), _dl2(s), _dl2(t)
            phi = np.array([Ls[a] * Lt[b] for b in range(3) for a in range(3)])
            px = np.array([dLs[a] * Lt[b] for b in range(3) for a in range(3)]) / hx
            py = np.array([Ls[a] * dLt[b] for b in range(3) for a in range(3)]) / hy
            M1s, M1t = _l1(s), _l1(t)
            psi = np.array([M1s[a] * M1t[b] for b in range(2) for a in range(2)])
            for n in range(9):
                for m in range(9):
                    A[2 * m, 2 * n] += w * nu * (2 * px[n] * px[m] + py[n] * py[m])
                    A[2 * m + 1, 2 * n + 1] += w * nu * (2 * py[n] * py[m] + px[n] * px[m])
                    A[2 * m + 1, 2 * n] += w * nu * py[n] * px[m]
                    A[2 * m, 2 * n + 1] += w * nu * px[n] * py[m]
            for q in range(4):
                for n in range(9):
                    B[q, 2 * n] -= w * px[n] * psi[q]
                    B[q, 2 * n + 1] -= w * py[n] * psi[q]
    return A, B


# triangles of one rectangle, as (a, b) corners on its 3x3 node grid (node
# 3*b + a at (a hx/2, b hy/2)); "/" cuts along (0,0)-(2,2), "\\" along (2,0)-(0,2)
_TRIANGLES = {"/": (((0, 0), (2, 0), (2, 2)), ((0, 0), (2, 2), (0, 2))),
              "\\": (((0, 0), (2, 0), (0, 2)), ((2, 0), (2, 2), (0, 2)))}
# edge-midpoint rule on a triangle: barycentric points, weights times |T|
_TRI_RULE = (np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]]), np.full(3, 1.0 / 3.0))


def diagonal(ex, ey, nx, ny):
    """Cut of element (ex, ey) of an nx x ny subdomain for the P2-P1 pair."""
    corner = (ex == nx - 1 and ey == 0) or (ex == 0 and ey == ny - 1)
    return "\\" if corner else "/"


def _pressure_node(a, b):
    """Q1/P1 pressure node of the rectangle corner at (a, b) on its node grid."""
    return 2 * (b // 2) + a // 2


def element_matrices_p2p1(hx, hy, nu, diag):
    """P2-P1 blocks of one rectangle cut into two triangles, in the layout of
    element_matrices: 18x18 velocity block and 4x18 divergence block.

    On a triangle with barycentric coordinates l_0, l_1, l_2 the P2 basis is
    l_i (2 l_i - 1) at vertex i and 4 l_i l_j at the midpoint of edge ij;
    the P1 pressure basis is l_i."""
    A = np.zeros((18, 18))
    B = np.zeros((4, 18))
    pts, wts = _TRI_RULE
    for tri in _TRIANGLES[diag]:
        xy = np.array([[a * hx / 2.0, b * hy / 2.0] for a, b in tri])
        # gradients of the barycentric coordinates: rows of the inverse of
        # [[1, 1, 1], [x_0, x_1, x_2], [y_0, y_1, y_2]] (first column dropped)
        T = np.vstack([np.ones(3), xy.T])
        G = np.linalg.inv(T)[:, 1:]          # G[i] = grad l_i
        area = 0.5 * abs(np.linalg.det(T))
        vnode = [3 * b + a for a, b in tri]
        enode = {(i, j): 3 * ((tri[i][1] + tri[j][1]) // 2) + (tri[i][0] + tri[j][0]) // 2
                 for i, j in ((0, 1), (1, 2), (0, 2))}
        pnode = [_pressure_node(a, b) for a, b in tri]
        for lam, w in zip(pts, wts * area):
            nodes, grads = [], []
            for i in range(3):
                nodes.append(vnode[i])
                grads.append((4.0 * lam[i] - 1.0) * G[i])
            for (i, j), nd in enode.items():
                nodes.append(nd)
                grads.append(4.0 * (lam[i] * G[j] + lam[j] * G[i]))
            for m, gm in zip(nodes, grads):
                for n, gn in zip(nodes, grads):
                    A[2 * m, 2 * n] += w * nu * (2 * gn[0] * gm[0] + gn[1] * gm[1])
                    A[2 * m + 1, 2 * n + 1] += w * nu * (2 * gn[1] * gm[1] + gn[0] * gm[0])
                    A[2 * m + 1, 2 * n] += w * nu * gn[1] * gm[0]
                    A[2 * m, 2 * n + 1] += w * nu * gn[0] * gm[1]
                for i in range(3):
                    B[pnode[i], 2 * m] -= w * gm[0] * lam[i]
                    B[pnode[i], 2 * m + 1] -= w * gm[1] * lam[i]
    return A, B


def stokes_element(layout):
    """'q2q1' (rectangles) or 'p2p1' (triangles) from the problem's discretization."""
    el = layout.prob.get("discretization", {}).get("stokes", "q2q1")
    if el not in ("q2q1", "p2p1"):
        raise ValueError("unknown Stokes element %r" % el)
    return el


class StokesLocal:
    """Local Q2-Q1 or P2-P1 operator of one Stokes subdomain."""

    def __init__(self, layout, i):
        self.layout, self.i = layout, i
        s = layout.subs[i]
        nx, ny = s["n"]
        hx, hy = s["h"]
        x0, x1, y0, y1 = s["rect"]
        ph = layout.phys
        nu = float(ph["nu_s"])
        self.nx, self.ny, self.hx, self.hy = nx, ny, hx, hy
        self.nnx, self.nny = 2 * nx + 1, 2 * ny + 1
        self.nvel = 2 * self.nnx * self.nny
        self.npre = (nx + 1) * (ny + 1)
        self.element = stokes_element(layout)
        if self.element == "q2q1":
            blocks = dict.fromkeys(("/", "\\"), element_matrices(hx, hy, nu))
        else:
            blocks = {d: element_matrices_p2p1(hx, hy, nu, d) for d in ("/", "\\")}
        rows, cols, vals, brow, bcol, bval = [], [], [], [], [], []
        for ey in range(ny):
            for ex in range(nx):
                Ae, Be = blocks[diagonal(ex, ey, nx, ny)]
                nodes = [(2 * ey + b) * self.nnx + 2 * ex + a for b in range(3) for a in range(3)]
                dofs = np.array([[2 * n, 2 * n + 1] for n in nodes]).ravel()
                pn = np.array([(ey + b) * (nx + 1) + ex + a for b in range(2) for a in range(2)])
                rr, cc = np.meshgrid(dofs, dofs, indexing="ij")
                rows.append(rr.ravel())
                cols.append(cc.ravel())
                vals.append(Ae.ravel())
                rr, cc = np.meshgrid(pn, dofs, indexing="ij")
                brow.append(rr.ravel())
                bcol.append(cc.ravel())
                bval.append(Be.ravel())
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.nvel, self.nvel)).tocsr()
        B = sp.coo_matrix((np.concatenate(bval), (np.concatenate(brow), np.concatenate(bcol))),
                          shape=(self.npre, self.nvel)).tocsr()
        # sides: classify fine edges; BJS and mortar traces
        self.sides = {}
        dirichlet_nodes = set()
        bjs_rows, bjs_cols, bjs_vals = [], [], []
        coef = bjs_coefficient(nu, float(ph["alpha"]), float(ph["k_bjs"]))
        R = layout.sub_dofs[i].size
        self.R = R
        Q = np.zeros((R, self.nvel))
        sign = layout.sub_sign[i]
        for side in ("bottom", "top", "left", "right"):
            if side in ("bottom", "top"):
                iy = 0 if side == "bottom" else self.nny - 1
                nodes = [iy * self.nnx + k for k in range(self.nnx)]
                tcoord = [x0 + 0.5 * k * hx for k in range(self.nnx)]
                h, nel = hx, nx
                normal = (0.0, -1.0) if side == "bottom" else (0.0, 1.0)
                tang = 0
            else:
                ix = 0 if side == "left" else self.nnx - 1
                nodes = [k * self.nnx + ix for k in range(self.nny)]
                tcoord = [y0 + 0.5 * k * hy for k in range(self.nny)]
                h, nel = hy, ny
                normal = (-1.0, 0.0) if side == "left" else (1.0, 0.0)
                tang = 1
            for e in range(nel):
                t0 = tcoord[2 * e]
                t1 = t0 + h
                f = layout.iface_at(i, side, 0.5 * (t0 + t1))
                enodes = nodes[2 * e: 2 * e + 3]
                if f is None:
                    dirichlet_nodes.update(enodes)
                    continue
                base = layout.local_index(i, f, 0)
                for a in range(3):
                    g = (lambda tt, a=a, t0=t0: _l2((tt - t0) / h)[a])
                    ints = f.node_integrals(t0, t1, g)
                    for nd in range(f.nnode):
                        if ints[nd] == 0.0:
                            continue
                        if f.kind == "ss":
                            for c in range(2):
                                q = base + 2 * nd + c
                                Q[q, 2 * enodes[a] + c] += sign[q] * ints[nd]
                        else:
                            q = base + nd
                            for c in range(2):
                                if normal[c] != 0.0:
                                    Q[q, 2 * enodes[a] + c] += normal[c] * ints[nd]
                if f.kind == "sd":
                    # BJS: coef * int u_tau v_tau on this fine edge
                    me = bjs_edge_mass(coef, h)
                    for a in range(3):
                        for b in range(3):
                            bjs_rows.append(2 * enodes[a] + tang)
                            bjs_cols.append(2 * enodes[b] + tang)
                            bjs_vals.append(me[a, b])
        if bjs_vals:
            A = A + sp.coo_matrix((bjs_vals, (bjs_rows, bjs_cols)), shape=(self.nvel, self.nvel)).tocsr()
        self.A, self.B, self.Q = A, B, Q
        dd = np.array(sorted(dirichlet_nodes), dtype=np.int64)
        self.dir_dofs = np.sort(np.concatenate([2 * dd, 2 * dd + 1])) if dd.size else np.zeros(0, np.int64)
        mask = np.ones(self.nvel, dtype=bool)
        mask[self.dir_dofs] = False
        self.free = np.nonzero(mask)[0]
        self.floating = layout.is_floating(i)
        self.uD = np.zeros(self.nvel)
        inflow = ph["inflow"]
        # outer velocity (u_x, u_y) = (inflow_x + shear y, inflow_y); shear = 0
        # gives the constant inflow of the configurations
        shear = float(ph.get("inflow_shear", 0.0))
        ynode = y0 + 0.5 * hy * (dd // self.nnx)
        self.uD[2 * dd] = inflow[0] + shear * ynode
        self.uD[2 * dd + 1] = inflow[1]
        # kernel of a~_i for floating subdomains: rigid motions left free by BJS
        self.Z = None
        if self.floating:
            self.Z = self._kernel(A, x0, x1, y0, y1)
        self._build_solver()

    def _kernel(self, A, x0, x1, y0, y1):
        X = np.array([x0 + 0.5 * k * self.hx for k in range(self.nnx)])
        Y = np.array([y0 + 0.5 * k * self.hy for k in range(self.nny)])
        XX, YY = np.meshgrid(X, Y)
        xc, yc = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
        rig = np.zeros((self.nvel, 3))
        rig[0::2, 0] = 1.0
        rig[1::2, 1] = 1.0
        rig[0::2, 2] = -(YY.ravel() - yc)
        rig[1::2, 2] = XX.ravel() - xc
        G = rig.T @ (A @ rig)
        w, V = np.linalg.eigh(G)
        keep = w < 1e-10 * max(1.0, np.abs(w).max())
        Z = rig @ V[:, keep]
        # orthonormal columns in the Euclidean coefficient inner product
        Zq, _ = np.linalg.qr(Z)
        return Zq

    def _build_solver(self):
        fr = self.free
        Af = self.A[fr][:, fr]
        Bf = self.B[:, fr]
        blocks = [[Af, Bf.T], [Bf, None]]
        if self.floating:
            Zf = sp.csr_matrix(self.Z[fr])
            blocks = [[Af, Bf.T, Zf], [Bf, None, None], [Zf.T, None, None]]
        K = sp.bmat(blocks, format="csc")
        self.nf = fr.size
        self._K = K.tocsr()
        self._lu = spla.splu(K)
        self._n = K.shape[0]

    def solve(self, load_vel, div_rhs=None):
        """Solve the local saddle problem for a velocity load on the free DOFs.

        Returns (u_free_values, p).  For floating subdomains the load is
        replaced by its compatible part and u is orthogonal to Z_i.
        """
        rhs = np.zeros(self._n)
        rhs[:self.nf] = load_vel
        if div_rhs is not None:
            rhs[self.nf:self.nf + self.npre] = div_rhs
        x = self._lu.solve(rhs)
        # one step of iterative refinement: the sparse LU of the saddle matrix
        # alone leaves rounding errors near 1e-9 in the pressure on 32x32
        # meshes; the refined x is the discrete solution to near machine precision
        x = x + self._lu.solve(rhs - self._K @ x)
        return x[:self.nf], x[self.nf:self.nf + self.npre]

    def star(self, lam_local):
        """u*(lambda), p*(lambda): zero outer data, interface load -<lambda, v>."""
        load = -(self.Q.T @ np.asarray(lam_local, dtype=np.float64))
        uf, p = self.solve(load[self.free])
        u = np.zeros(self.nvel)
        u[self.free] = uf
        return u, p

    def bar(self):
        """Complementary problem: outer velocity data, zero interface stress, f = 0."""
        rhs_u = -(self.A @ self.uD)[self.free]
        rhs_p = -(self.B @ self.uD)
        uf, p = self.solve(rhs_u, rhs_p)
        u = self.uD.copy()
        u[self.free] = uf
        return u, p

    def response(self, lam_local):
        u, _ = self.star(lam_local)
        return -(self.Q @ u)

    def basis(self):
        S = np.zeros((self.R, self.R))
        for j in range(self.R):
            e = np.zeros(self.R)
            e[j] = 1.0
            S[:, j] = self.response(e)
        return S

    def g_local(self):
        """Local contribution Q_i u_bar to the right-hand side g_H (eq. operatorform)."""
        u, _ = self.bar()
        return self.Q @ u

    def kernel_trace(self):
        """Q_i Z_i: the columns of the FETI matrix G restricted to Gamma_i."""
        return self.Q @ self.Z
