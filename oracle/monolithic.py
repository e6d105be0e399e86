"""The fully discrete coupled problem solved directly (oracle).

Section 4, eqs. (fullydisc1-2) for one realization: all subdomain velocity
and pressure unknowns plus the mortar multiplier lambda in one sparse saddle
system built from the forms of Section 3.2,
  a~(u, v) + b~(v, p) + b~_Lambda(v, lambda) = (f, v)
  b~(u, w) = -(q_d, w)
  b~_Lambda(u, mu) = 0,
solved by sparse LU.  The Darcy part is kept in its mixed RT0-Q0 form
(velocities on edges with the trapezoidal mass, or with the exactly
integrated mass that couples the two opposite faces of a cell), so this
path shares neither the cell-centred nor the hybridized elimination of the
domain-decomposition solvers; agreement of the two pins the interface
reduction of Section 5.1.  Floating Stokes
subdomains need no special treatment here.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .stokes import StokesLocal


def rt0_pair_mass(exact):
    """Velocity mass of the two opposite faces of a unit cell with K = nu = 1,
    in +x / +y oriented normal velocities: int phi_a phi_b for the linear
    shape functions (1 - s) and s, or its trapezoidal (vertex) rule."""
    if exact:
        return np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
    return np.array([[0.5, 0.0], [0.0, 0.5]])


def darcy_mixed(layout, i, K):
    """RT0-Q0 blocks of Darcy subdomain i: (mass, B, Q, rhs_u, kept edges)."""
    s = layout.subs[i]
    nx, ny = s["n"]
    hx, hy = s["h"]
    nu = float(layout.phys["nu_d"])
    area = hx * hy
    nv = (nx + 1) * ny
    ne = nv + nx * (ny + 1)
    N = nx * ny
    pm = rt0_pair_mass(layout.prob.get("discretization", {}).get("darcy", "trapezoidal") == "exact")
    mr, mc, mv = [], [], []
    for iy in range(ny):
        for ix in range(nx):
            c = iy * nx + ix
            for pair in ((iy * (nx + 1) + ix, iy * (nx + 1) + ix + 1), (nv + iy * nx + ix, nv + (iy + 1) * nx + ix)):
                for a in range(2):
                    for b in range(2):
                        mr.append(pair[a])
                        mc.append(pair[b])
                        mv.append(nu * area / K[c] * pm[a, b])
    mass = sp.coo_matrix((mv, (mr, mc)), shape=(ne, ne)).tocsr()
    B = sp.lil_matrix((N, ne))
    for iy in range(ny):
        for ix in range(nx + 1):
            e = iy * (nx + 1) + ix
            for cx, sgn in ((ix - 1, -1.0), (ix, 1.0)):
                if 0 <= cx < nx:
                    c = iy * nx + cx
                    # cell on the left sees outward +x: -(div phi, 1_c) = -|e|
                    B[c, e] = sgn * hy
    for iy in range(ny + 1):
        for ix in range(nx):
            e = nv + iy * nx + ix
            for cy, sgn in ((iy - 1, -1.0), (iy, 1.0)):
                if 0 <= cy < ny:
                    c = cy * nx + ix
                    B[c, e] = sgn * hx
    R = layout.sub_dofs[i].size
    Q = np.zeros((R, ne))
    rhs = np.zeros(ne)
    keep = np.ones(ne, dtype=bool)
    pb = float(layout.phys["p_bottom"])
    for be in layout.darcy_boundary(i):
        e = be["edge"]
        if be["kind"] == "noflow":
            keep[e] = False
        elif be["kind"] == "dirichlet":
            rhs[e] = -pb * be["length"] * be["sgn"]
        else:
            f = layout.ifaces[be["iface"]]
            ints = f.node_integrals(be["t0"], be["t1"])
            base = layout.local_index(i, f, 0)
            Q[base:base + f.ndof, e] += be["sgn"] * ints
    return mass, B.tocsr(), Q, rhs, np.nonzero(keep)[0]


def system(layout, darcy_K, stokes=None):
    """Assemble the coupled saddle system of one realization.

    Returns (Bd, Qall, rhs, info): the block-diagonal subdomain matrix, the
    mortar coupling rows b~_Lambda, the right-hand side and the block layout.
    """
    L = layout
    M = L.M
    blocks_diag = []
    coup = []   # per block: (Q columns on its unknowns, offset)
    rhs_parts = []
    lam_rhs = np.zeros(M)
    info = []
    if stokes is None:
        stokes = {}
    for i in range(L.nsub):
        if L.subs[i]["type"] == "stokes":
            st = stokes.get(i) or StokesLocal(L, i)
            fr = st.free
            Af = st.A[fr][:, fr]
            Bf = st.B[:, fr]
            blk = sp.bmat([[Af, Bf.T], [Bf, None]], format="csr")
            ru = -(st.A @ st.uD)[fr]
            rp = -(st.B @ st.uD)
            Qfull = np.zeros((M, st.nvel))
            Qfull[L.sub_dofs[i]] = st.Q
            lam_rhs -= Qfull @ st.uD
            Qblk = sp.hstack([sp.csr_matrix(Qfull[:, fr]), sp.csr_matrix((M, st.npre))])
            blocks_diag.append(blk)
            coup.append(Qblk)
            rhs_parts.append(np.concatenate([ru, rp]))
            info.append(("stokes", i, st, fr.size, st.npre))
        else:
            K = darcy_K[i]
            mass, B, Q, ru, keep = darcy_mixed(L, i, K)
            Mk = mass[keep][:, keep]
            Bk = B[:, keep]
            blk = sp.bmat([[Mk, Bk.T], [Bk, None]], format="csr")
            Qfull = np.zeros((M, mass.shape[0]))
            Qfull[L.sub_dofs[i]] = Q
            Qblk = sp.hstack([sp.csr_matrix(Qfull[:, keep]), sp.csr_matrix((M, B.shape[0]))])
            blocks_diag.append(blk)
            coup.append(Qblk)
            rhs_parts.append(np.concatenate([ru[keep], np.zeros(B.shape[0])]))
            info.append(("darcy", i, keep, mass.shape[0], B.shape[0]))
    Bd = sp.block_diag(blocks_diag, format="csr")
    Qall = sp.hstack(coup, format="csr")
    rhs = np.concatenate(rhs_parts + [lam_rhs])
    return Bd, Qall, rhs, info


def solve(layout, darcy_K, stokes=None):
    """Direct solve of one realization.

    darcy_K maps Darcy subdomain index -> cell permeabilities.  Returns a dict
    with the fields named in oracle.methods.FIELDS.
    """
    Bd, Qall, rhs, info = system(layout, darcy_K, stokes)
    K = sp.bmat([[Bd, Qall.T], [Qall, None]], format="csc")
    x = spla.splu(K).solve(rhs)
    lam = x[Bd.shape[0]:]
    out = {"lambda": lam}
    off = 0
    dp, du, su, sp_ = [], [], [], []
    for kind, i, a, b, c in info:
        if kind == "stokes":
            st, nf, npre = a, b, c
            u = st.uD.copy()
            u[st.free] = x[off:off + nf]
            su.append(u)
            sp_.append(x[off + nf:off + nf + npre])
            off += nf + npre
        else:
            keep, ne, N = a, b, c
            u = np.zeros(ne)
            u[keep] = x[off:off + keep.size]
            du.append(u)
            dp.append(x[off + keep.size:off + keep.size + N])
            off += keep.size + N
    out["darcy_p"] = np.concatenate(dp) if dp else np.zeros(0)
    out["darcy_u"] = np.concatenate(du) if du else np.zeros(0)
    out["stokes_u"] = np.concatenate(su) if su else np.zeros(0)
    out["stokes_p"] = np.concatenate(sp_) if sp_ else np.zeros(0)
    return out
