"""Interface problem and its Krylov solution (oracle).

Section 5.1, eqs. (interface) and (operatorform): the coupled problem
reduces to S_H lambda = g_H with S_H = sum_i S_{H,i} (each local operator
acting on the restriction of lambda to Gamma_i) and g_H given by the
complementary solutions.  s_H is symmetric positive definite and is solved
by CG.  Floating Stokes subdomains add the FETI coarse problem
  [S -G; -G^T 0] [lambda; alpha] = [g; -e]
whose lambda part is found by CG projected with P = I - G (G^T G)^{-1} G^T.

Reading of the CG (the paper gives none): lambda_0 = 0 (or the FETI
particular solution), no preconditioner, stop when ||r_k||_2 <= rtol ||r_0||_2
on mortar coefficients (r_0 = g, or P g when FETI projects), at most
max_iter iterations.
"""
import numpy as np


def assemble(layout, S_local):
    """Dense S_H = sum_i R_i^T S_{H,i} R_i."""
    M = layout.M
    S = np.zeros((M, M))
    for i, Si in enumerate(S_local):
        d = layout.sub_dofs[i]
        S[np.ix_(d, d)] += Si
    return S


def restrict(layout, i, lam):
    return np.asarray(lam)[layout.sub_dofs[i]]


def cg(apply, g, rtol=1e-8, max_iter=None, G=None, e=None):
    """Plain (optionally FETI-projected) CG.

    apply(x) returns S x; G (M x q) and e (q) describe the FETI constraint
    G^T lambda = e.  Returns (lambda, iterations, relres, converged).
    """
    g = np.asarray(g, dtype=np.float64)
    n = g.size
    if max_iter is None:
        max_iter = 10 * n
    if G is not None and G.shape[1] > 0:
        GtG = G.T @ G
        proj = lambda v: v - G @ np.linalg.solve(GtG, G.T @ v)
        lam0 = G @ np.linalg.solve(GtG, e) if e is not None else np.zeros(n)
    else:
        proj = lambda v: v
        lam0 = np.zeros(n)
    lam = lam0.copy()
    r = proj(g - apply(lam)) if np.any(lam0) else proj(g.copy())
    gnorm = np.linalg.norm(r)
    if gnorm == 0.0:
        return lam, 0, 0.0, True
    p = r.copy()
    rr = r @ r
    it = 0
    if np.sqrt(rr) <= rtol * gnorm:
        return lam, 0, np.sqrt(rr) / gnorm, True
    while it < max_iter:
        w = proj(apply(p))
        pw = p @ w
        if not pw > 0.0:
            return lam, it, np.sqrt(rr) / gnorm, False
        a = rr / pw
        lam += a * p
        r -= a * w
        rr_new = r @ r
        it += 1
        if np.sqrt(rr_new) <= rtol * gnorm:
            return lam, it, np.sqrt(rr_new) / gnorm, True
        p = r + (rr_new / rr) * p
        rr = rr_new
    return lam, it, np.sqrt(rr) / gnorm, False


def feti_alpha(G, S_apply, lam, g):
    """Kernel coefficients alpha = (G^T G)^{-1} G^T (S lambda - g)."""
    return np.linalg.solve(G.T @ G, G.T @ (S_apply(lam) - g))
