"""Methods S1, S2, S3 and the statistical moments (oracle).

Section 5.2 (Method S1: subdomain solves inside every CG iteration),
Section 5.3 (Method S2: a deterministic multiscale flux basis per global
realization; S_{H,i} lambda = sum_j c_i^j phi^j) and Section 5.4 (Method S3:
a stochastic basis for every local realization of each Darcy subdomain's KL
region, computed before the collocation loop; Stokes subdomains have one
local realization).  Moments follow Section 2 (E and Var = E[xi^2] - E[xi]^2)
with the collocation weights of Section 4 (w_k = int L_k rho).

Solve counters follow eqs. (S1-cost), (S2-cost), (S3-cost) plus the two
extra solves per realization (right-hand side and recovery) that Section
5.4 names.

Fields whose moments are returned (reading; the paper plots velocity and
pressure means and variances):
  lambda    mortar coefficients (M)
  darcy_p   Darcy cell pressures, subdomain by subdomain, cells row-major
  darcy_u   Darcy RT0 normal velocities (+x / +y), subdomain by subdomain
  stokes_u  Stokes Q2 nodal velocities (2 per node, x then y), all nodes
  stokes_p  Stokes Q1 nodal pressures
"""
import numpy as np

from . import interface as itf
from .collocation import Grid
from .darcy import make_darcy_local
from .geometry import Layout
from .kl import cell_centres, region_field
from .stokes import StokesLocal

FIELDS = ("lambda", "darcy_p", "darcy_u", "stokes_u", "stokes_p")


def _map(fn, items, threads, progress=None):
    """fn over independent items, in order; threads > 1 only overlaps the
    sparse factorizations (SuperLU releases the GIL), the arithmetic is the
    same.  progress(item) is called as each item finishes."""
    def run(x):
        y = fn(x)
        if progress is not None:
            progress(x)
        return y
    if threads <= 1:
        return [run(x) for x in items]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(run, items))


class Oracle:
    def __init__(self, prob, threads=1, progress=None):
        self.prob = prob
        self.threads = threads
        self.progress = progress
        self.L = Layout(prob)
        self.grid = Grid(prob["regions"], prob["rule"])
        L = self.L
        self.stokes_ids = [i for i in range(L.nsub) if L.subs[i]["type"] == "stokes"]
        self.darcy_ids = [i for i in range(L.nsub) if L.subs[i]["type"] == "darcy"]
        self.stokes = dict(zip(self.stokes_ids, _map(lambda i: StokesLocal(L, i), self.stokes_ids, threads,
                                                           progress)))
        self.phi = {}
        for i in self.darcy_ids:
            reg = L.regions[L.subs[i]["region"]]
            self.phi[i] = region_field(reg, cell_centres(L.subs[i]))
        # FETI matrix G (global mortar x kernel modes) and its constraint data e
        cols = []
        for i in self.stokes_ids:
            st = self.stokes[i]
            if st.floating:
                Gi = st.kernel_trace()
                for c in range(Gi.shape[1]):
                    col = np.zeros(L.M)
                    col[L.sub_dofs[i]] = Gi[:, c]
                    cols.append(col)
        self.G = np.stack(cols, axis=1) if cols else np.zeros((L.M, 0))
        self.e = np.zeros(self.G.shape[1])
        self.g_stokes = np.zeros(L.M)
        self.stokes_bar = {}
        for i in self.stokes_ids:
            u, p = self.stokes[i].bar()
            self.stokes_bar[i] = (u, p)
            self.g_stokes[L.sub_dofs[i]] += self.stokes[i].Q @ u
        self.counters = {}
        self._stokes_S = None

    # ---- per realization data -------------------------------------------------
    def region_point(self, y_global, r):
        o = self.grid.dim_off
        return np.asarray(y_global)[o[r]:o[r + 1]]

    def darcy_K(self, i, y_region):
        reg = self.L.regions[self.L.subs[i]["region"]]
        return np.exp(float(reg["mean_logk"]) + np.asarray(y_region) @ self.phi[i])

    def darcy_local(self, i, y_global):
        r = self.L.subs[i]["region"]
        return make_darcy_local(self.L, i, self.darcy_K(i, self.region_point(y_global, r)))

    def g_vector(self, darcy_locals):
        g = self.g_stokes.copy()
        pb = float(self.L.phys["p_bottom"])
        if pb != 0.0:
            for i, dl in darcy_locals.items():
                _, uout = dl.solve(np.zeros(dl.R), p_outer=pb)
                g[self.L.sub_dofs[i]] += dl.avg.T @ uout
        return g

    def stokes_basis(self):
        if self._stokes_S is None:
            self._stokes_S = dict(zip(self.stokes_ids,
                                      _map(lambda i: self.stokes[i].basis(), self.stokes_ids, self.threads,
                                           self.progress)))
        return self._stokes_S

    def _count(self, i, n):
        self.counters[i] = self.counters.get(i, 0) + n

    # ---- recovery ----------------------------------------------------------
    def recover(self, lam, darcy_locals, S_apply, g):
        """Fine-scale fields u = u*(lambda) + u_bar (+ Z alpha) for one realization."""
        L = self.L
        out = {"lambda": lam.copy()}
        alpha = None
        if self.G.shape[1]:
            alpha = itf.feti_alpha(self.G, S_apply, lam, g)
        dp, du = [], []
        pb = float(L.phys["p_bottom"])
        for i in self.darcy_ids:
            dl = darcy_locals[i]
            ll = lam[L.sub_dofs[i]]
            p, _ = dl.solve(ll, p_outer=pb)
            dp.append(p)
            du.append(dl.velocities(p, ll, p_outer=pb))
        su, spr = [], []
        col = 0
        for i in self.stokes_ids:
            st = self.stokes[i]
            u, p = st.star(lam[L.sub_dofs[i]])
            ub, pbar = self.stokes_bar[i]
            u = u + ub
            p = p + pbar
            if st.floating:
                k = st.Z.shape[1]
                u = u + st.Z @ alpha[col:col + k]
                col += k
            su.append(u)
            spr.append(p)
        out["darcy_p"] = np.concatenate(dp) if dp else np.zeros(0)
        out["darcy_u"] = np.concatenate(du) if du else np.zeros(0)
        out["stokes_u"] = np.concatenate(su) if su else np.zeros(0)
        out["stokes_p"] = np.concatenate(spr) if spr else np.zeros(0)
        return out

    # ---- one realization through each method -----------------------------------
    def _solve_with(self, S_apply, g, rtol, max_iter):
        return itf.cg(S_apply, g, rtol=rtol, max_iter=max_iter,
                      G=self.G if self.G.shape[1] else None, e=self.e if self.G.shape[1] else None)

    def realization_S1(self, l, rtol=1e-8, max_iter=None):
        L = self.L
        y = self.grid.points[l]
        dls = {i: self.darcy_local(i, y) for i in self.darcy_ids}
        nsolve = [0]

        def apply(x):
            nsolve[0] += 1
            out = np.zeros(L.M)
            for i in self.darcy_ids:
                out[L.sub_dofs[i]] += dls[i].response(x[L.sub_dofs[i]])
            for i in self.stokes_ids:
                out[L.sub_dofs[i]] += self.stokes[i].response(x[L.sub_dofs[i]])
            return out

        g = self.g_vector(dls)
        lam, it, rel, ok = self._solve_with(apply, g, rtol, max_iter)
        napply = nsolve[0]
        fields = self.recover(lam, dls, apply, g)
        for i in range(L.nsub):
            self._count(i, napply + 2)
        return fields, it, rel, ok

    def realization_S2(self, l, rtol=1e-8, max_iter=None):
        return self.point_S2(self.grid.points[l], rtol=rtol, max_iter=max_iter)

    def point_S2(self, y, rtol=1e-8, max_iter=None):
        """Method S2 (Section 5.3) at one point y of the stochastic space, on
        the collocation grid or not: every S_{H,i} is built from the local
        problems of y's own KL field (eq. KLapprox), then CG on S_H."""
        L = self.L
        y = np.asarray(y, dtype=np.float64)
        dls = {i: self.darcy_local(i, y) for i in self.darcy_ids}
        S_loc = [None] * L.nsub
        for i in self.darcy_ids:
            S_loc[i] = dls[i].basis()
        for i in self.stokes_ids:
            S_loc[i] = self.stokes[i].basis()
        for i in range(L.nsub):
            self._count(i, L.sub_dofs[i].size + 2)
        S = itf.assemble(L, S_loc)
        g = self.g_vector(dls)
        lam, it, rel, ok = self._solve_with(lambda x: S @ x, g, rtol, max_iter)
        return self.recover(lam, dls, lambda x: S @ x, g), it, rel, ok

    def stochastic_basis(self):
        """Method S3 pre-computation loop: S_{H,i}^{(k)} for every local realization k."""
        L = self.L
        table = {}
        for i in self.darcy_ids:
            r = L.subs[i]["region"]
            ylocs = self.grid.local_points(r)
            for k in range(ylocs.shape[0]):
                dl = make_darcy_local(L, i, self.darcy_K(i, ylocs[k]))
                table[(i, k)] = dl.basis()
            self._count(i, L.sub_dofs[i].size * ylocs.shape[0])
        for i, S in self.stokes_basis().items():
            table[(i, 0)] = S
            self._count(i, L.sub_dofs[i].size)
        self.s3_table = table
        return table

    def realization_S3(self, l, rtol=1e-8, max_iter=None):
        L = self.L
        if not hasattr(self, "s3_table"):
            self.stochastic_basis()
        kl = self.grid.g2l[l]
        S_loc = [None] * L.nsub
        for i in self.darcy_ids:
            S_loc[i] = self.s3_table[(i, int(kl[L.subs[i]["region"]]))]
        for i in self.stokes_ids:
            S_loc[i] = self.s3_table[(i, 0)]
        S = itf.assemble(L, S_loc)
        y = self.grid.points[l]
        dls = {i: self.darcy_local(i, y) for i in self.darcy_ids}
        g = self.g_vector(dls)
        lam, it, rel, ok = self._solve_with(lambda x: S @ x, g, rtol, max_iter)
        for i in range(L.nsub):
            self._count(i, 2)
        return self.recover(lam, dls, lambda x: S @ x, g), it, rel, ok

    # ---- collocation loop -------------------------------------------------------
    def run(self, method="S3", indices=None, weights=None, rtol=1e-8, max_iter=None):
        """Collocation loop; returns (moments {field: (mean, var)}, per-realization info)."""
        self.counters = {}
        if method == "S3":
            self.stochastic_basis()
        fn = {"S1": self.realization_S1, "S2": self.realization_S2, "S3": self.realization_S3}[method]
        idx = range(self.grid.nreal) if indices is None else indices
        w = self.grid.weights if weights is None else None
        acc1, acc2, info = {}, {}, []
        for n, l in enumerate(idx):
            wl = float(w[l]) if weights is None else float(weights[n])
            fields, it, rel, ok = fn(l, rtol=rtol, max_iter=max_iter)
            info.append({"l": l, "iters": it, "relres": rel, "ok": ok, "lambda": fields["lambda"]})
            for k, v in fields.items():
                if k not in acc1:
                    acc1[k] = np.zeros_like(v)
                    acc2[k] = np.zeros_like(v)
                acc1[k] += wl * v
                acc2[k] += wl * v * v
        mom = {k: (acc1[k], acc2[k] - acc1[k] ** 2) for k in acc1}
        return mom, info
