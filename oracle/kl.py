"""Multi-region KL expansion of the log-permeability (oracle).

Section 2.1 (eqs. Fred, KL, KLapprox): each KL region carries its own
truncated expansion Y' = sum_j xi_j sqrt(lambda_j) f_j(x), with eigenpairs of
the covariance kernel; Section 6 (eq. covariance) fixes the separable
exponential kernel sigma^2 exp(-|dx1|/eta1 - |dx2|/eta2).

Readings (the paper solves the Fredholm problem "numerically" and does not
say which modes are kept):
* the covariance amplitude is sigma^2;
* the kernel factorises, so the 2-D eigenpairs are products of 1-D eigenpairs
  of exp(-|x - x'|/eta) on [-a, a] (a = half the region width), whose roots
  solve c - w tan(w a) = 0 (even modes) and w + c tan(w a) = 0 (odd modes),
  c = 1/eta, lambda = 2c / (w^2 + c^2);
* the N_term kept modes are the N_term largest products; ties go to the
  smaller a + b, then the smaller a;
* eigenfunctions are cos / sin about the region centre with positive
  amplitude; K is sampled at cell centres, K_c = exp(Y(x_c)).
A Nystrom discretisation of the 1-D kernel is provided as an independent
check of the closed form.
"""
import numpy as np
from scipy.optimize import brentq


def eig1d(a, eta, nmodes):
    """First nmodes 1-D eigenpairs, ordered by decreasing eigenvalue.

    Returns (lam[n], omega[n], parity[n] (0 even / 1 odd), norm[n]) where the
    eigenfunction is cos(w x)/norm (even) or sin(w x)/norm (odd) on [-a, a].
    """
    c = 1.0 / eta
    lam, om, par, nrm = [], [], [], []
    for n in range(nmodes):
        k = n // 2
        if n % 2 == 0:
            # c cos(w a) - w sin(w a) = 0  on  w a in (k pi, k pi + pi/2)
            f = lambda w: c * np.cos(w * a) - w * np.sin(w * a)
            lo, hi = k * np.pi / a, (k * np.pi + 0.5 * np.pi) / a
        else:
            # w cos(w a) + c sin(w a) = 0  on  w a in (k pi + pi/2, (k+1) pi)
            f = lambda w: w * np.cos(w * a) + c * np.sin(w * a)
            lo, hi = (k * np.pi + 0.5 * np.pi) / a, ((k + 1) * np.pi) / a
        eps = 1e-14 * (hi - lo) + 1e-300
        w = brentq(f, lo + eps if lo > 0 else 1e-300, hi - eps, xtol=1e-16, rtol=1e-15, maxiter=500)
        lam.append(2.0 * c / (w * w + c * c))
        om.append(w)
        par.append(n % 2)
        if n % 2 == 0:
            nrm.append(np.sqrt(a + np.sin(2.0 * w * a) / (2.0 * w)))
        else:
            nrm.append(np.sqrt(a - np.sin(2.0 * w * a) / (2.0 * w)))
    return np.array(lam), np.array(om), np.array(par), np.array(nrm)


def eval1d(x, om, par, nrm):
    x = np.asarray(x, dtype=np.float64)
    return (np.cos(om * x) if par == 0 else np.sin(om * x)) / nrm


def region_modes(region):
    """Kept 2-D modes of one KL region.

    Returns a list of dicts (a, b, lam2d) sorted by the selection rule, plus
    the 1-D tables for both directions.
    """
    x0, x1, y0, y1 = region["rect"]
    nt = int(region["nterm"])
    s2 = float(region["sigma2"])
    e1, e2 = [float(v) for v in region["eta"]]
    ax, ay = 0.5 * (x1 - x0), 0.5 * (y1 - y0)
    nm = nt + 1
    tx = eig1d(ax, e1, nm)
    ty = eig1d(ay, e2, nm)
    cand = []
    for a in range(nm):
        for b in range(nm):
            cand.append((-(s2 * tx[0][a] * ty[0][b]), a + b, a, b))
    cand.sort()
    modes = [{"a": c[2], "b": c[3], "lam": -c[0]} for c in cand[:nt]]
    return modes, tx, ty


def region_field(region, pts):
    """sqrt(lambda_t) f_t(x) for every kept mode t at points pts (nterm x npts)."""
    x0, x1, y0, y1 = region["rect"]
    xc, yc = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
    modes, tx, ty = region_modes(region)
    pts = np.asarray(pts, dtype=np.float64)
    out = np.zeros((len(modes), pts.shape[0]))
    for t, m in enumerate(modes):
        fa = eval1d(pts[:, 0] - xc, tx[1][m["a"]], tx[2][m["a"]], tx[3][m["a"]])
        fb = eval1d(pts[:, 1] - yc, ty[1][m["b"]], ty[2][m["b"]], ty[3][m["b"]])
        out[t] = np.sqrt(m["lam"]) * fa * fb
    return out


def cell_centres(sub):
    x0, x1, y0, y1 = sub["rect"]
    nx, ny = sub["n"]
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    X, Y = np.meshgrid(x0 + (np.arange(nx) + 0.5) * hx, y0 + (np.arange(ny) + 0.5) * hy)
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def darcy_permeability(layout, i, y_local):
    """K on the cells of Darcy subdomain i for the region-local point y_local.

    Y(x_c) = E[Y] + sum_t y_t sqrt(lambda_t) f_t(x_c)  (eq. KLapprox), K = exp(Y).
    """
    sub = layout.subs[i]
    reg = layout.regions[sub["region"]]
    phi = region_field(reg, cell_centres(sub))
    y = np.asarray(y_local, dtype=np.float64)
    return np.exp(float(reg["mean_logk"]) + y @ phi)


def nystrom1d(a, eta, n, nmodes):
    """Eigenvalues of exp(-|x-x'|/eta) on [-a, a] by the midpoint Nystrom rule."""
    h = 2.0 * a / n
    x = -a + (np.arange(n) + 0.5) * h
    Kmat = np.exp(-np.abs(x[:, None] - x[None, :]) / eta) * h
    ev = np.linalg.eigvalsh(Kmat)[::-1]
    return ev[:nmodes]
