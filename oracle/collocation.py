"""Stochastic collocation rules and global/local index maps (oracle).

Section 4: the 1-D rules are Gauss-Hermite for the N(0,1) density of each
xi_j (Section 2.1); the tensor grid (Section 4.1) takes the product of 1-D
rules in kappa order; the Smolyak grid (Section 4.2) combines tensor rules
over levels l_min <= |p| <= l_max with coefficients
(-1)^(l_max-|p|) binom(N-1, l_max-|p|) and 1-D rules with 2^(p+1)-1 points.

Readings:
* The printed H_m is the physicists' Hermite polynomial; the density is the
  standard normal, so the nodes used are the probabilists' ones and the
  weights sum to one (Golub-Welsch on the probabilists' recurrence).
* Node ids: tensor rules number nodes by ascending abscissa; sparse rules
  give 0 the id 0 and the other distinct abscissae (union over levels)
  ascending ids.  A grid point is its tuple of node ids; global points are
  sorted lexicographically by that tuple (for a tensor grid this is the
  mixed-radix order with the last dimension fastest).
* A region's local realizations are the distinct projections of the global
  points onto the region's dimensions, sorted lexicographically; the
  global->local table maps every global point to its projection's position
  (Step 4 of Method S3; the paper defers the algorithm to another work).
* Coincident sparse points are merged and their weights summed.
"""
import itertools
from math import comb

import numpy as np


def gauss_hermite(m):
    """Probabilists' Gauss-Hermite rule with m nodes; weights sum to one."""
    if m == 1:
        return np.array([0.0]), np.array([1.0])
    off = np.sqrt(np.arange(1, m, dtype=np.float64))
    J = np.diag(off, 1) + np.diag(off, -1)
    x, V = np.linalg.eigh(J)
    w = V[0, :] ** 2
    # enforce the exact symmetry of the rule
    x = 0.5 * (x - x[::-1])
    w = 0.5 * (w + w[::-1])
    if m % 2 == 1:
        x[m // 2] = 0.0
    return x, w / w.sum()


def sparse_level_points(p, growth):
    return (2 ** (p + 1) - 1) if growth == "paper" else (p + 1)


class Grid:
    """Global collocation points, weights and region-local index tables."""

    def __init__(self, regions, rule):
        self.nterm_r = [int(r["nterm"]) for r in regions]
        self.N = sum(self.nterm_r)
        self.dim_off = np.concatenate([[0], np.cumsum(self.nterm_r)]).astype(int)
        kind = rule["kind"]
        if kind == "tensor":
            self._tensor(rule)
        elif kind == "sparse":
            self._sparse(rule)
        else:
            raise ValueError("unknown rule kind")
        self.nreal = self.ids.shape[0]
        self.points = self.node_x[self.ids]
        self.local_ids, self.g2l = [], []
        for r in range(len(self.nterm_r)):
            sl = self.ids[:, self.dim_off[r]:self.dim_off[r + 1]]
            uniq, inv = np.unique(sl, axis=0, return_inverse=True)
            self.local_ids.append(uniq)
            self.g2l.append(inv.reshape(-1).astype(np.int64))
        self.g2l = np.stack(self.g2l, axis=1) if self.g2l else np.zeros((self.nreal, 0), np.int64)
        self.nlocal = [u.shape[0] for u in self.local_ids]

    def local_points(self, r):
        return self.node_x[self.local_ids[r]]

    def _tensor(self, rule):
        m = int(rule["m"])
        x, w = gauss_hermite(m)
        self.node_x = x
        ids = np.array(list(itertools.product(range(m), repeat=self.N)), dtype=np.int64)
        if self.N == 0:
            ids = np.zeros((1, 0), dtype=np.int64)
        self.ids = ids
        self.weights = np.prod(w[ids], axis=1) if self.N else np.ones(1)

    def _sparse(self, rule):
        L = int(rule["level"])
        growth = rule.get("growth", "paper")
        N = self.N
        rules = {}
        allx = []
        for p in range(L + 1):
            rules[p] = gauss_hermite(sparse_level_points(p, growth))
            allx.extend(rules[p][0].tolist())
        allx = np.array(allx)
        uniq = []
        for v in np.sort(allx):
            if not uniq or abs(v - uniq[-1]) > 1e-10:
                uniq.append(v)
        uniq = np.array(uniq)
        has0 = np.any(np.abs(uniq) < 1e-13)
        nz = [v for v in uniq if abs(v) >= 1e-13]
        node_x = ([0.0] if has0 else []) + nz
        self.node_x = np.array(node_x)

        def nid(v):
            return int(np.argmin(np.abs(self.node_x - v)))

        rule_ids = {p: [nid(v) for v in rules[p][0]] for p in rules}
        lmin = max(0, L - N + 1)
        acc = {}
        for tot in range(lmin, L + 1):
            coef = (-1) ** (L - tot) * comb(N - 1, L - tot)
            for p in _compositions(tot, N):
                lists = [list(zip(rule_ids[pk], rules[pk][1])) for pk in p]
                for combo in itertools.product(*lists):
                    key = tuple(c[0] for c in combo)
                    wv = coef * float(np.prod([c[1] for c in combo]))
                    acc[key] = acc.get(key, 0.0) + wv
        keys = sorted(acc.keys())
        self.ids = np.array(keys, dtype=np.int64).reshape(len(keys), N)
        self.weights = np.array([acc[k] for k in keys])


def _compositions(total, n):
    """All n-tuples of non-negative ints summing to total."""
    if n == 1:
        yield (total,)
        return
    for first in range(total + 1):
        for rest in _compositions(total - first, n - 1):
            yield (first,) + rest
