"""Pins of the KL part of the oracle (Section 2.1, eq. Fred; Section 6, eq. covariance)."""
import numpy as np
import pytest

from oracle import kl
from workloads import problem


@pytest.mark.parametrize("a,eta", [(0.25, 0.2), (0.5, 0.2), (0.25, 0.1), (0.5, 0.05), (0.25, 0.3)])
def test_closed_form_matches_nystrom(a, eta):
    lam, om, par, nrm = kl.eig1d(a, eta, 6)
    ny = kl.nystrom1d(a, eta, 2000, 6)
    assert np.allclose(lam, ny, rtol=2e-5, atol=0)
    assert np.all(np.diff(lam) < 0)


@pytest.mark.parametrize("a,eta", [(0.25, 0.2), (0.5, 0.1)])
def test_fredholm_equation_by_quadrature(a, eta):
    """int C(x, xb) f(x) dx = lambda f(xb), evaluated with fine Gauss quadrature."""
    lam, om, par, nrm = kl.eig1d(a, eta, 5)
    xg, wg = np.polynomial.legendre.leggauss(200)
    for xb in (-0.8 * a, -0.1 * a, 0.37 * a, 0.9 * a):
        for n in range(5):
            tot = 0.0
            for lo, hi in ((-a, xb), (xb, a)):  # split at the kink of the kernel
                x = 0.5 * (hi + lo) + 0.5 * (hi - lo) * xg
                tot += 0.5 * (hi - lo) * np.sum(wg * np.exp(-np.abs(x - xb) / eta)
                                                * kl.eval1d(x, om[n], par[n], nrm[n]))
            assert abs(tot - lam[n] * kl.eval1d(xb, om[n], par[n], nrm[n])) < 1e-11


def test_orthonormality():
    a, eta = 0.5, 0.2
    lam, om, par, nrm = kl.eig1d(a, eta, 6)
    xg, wg = np.polynomial.legendre.leggauss(400)
    x, w = a * xg, a * wg
    F = np.stack([kl.eval1d(x, om[n], par[n], nrm[n]) for n in range(6)])
    assert np.allclose((F * w) @ F.T, np.eye(6), atol=1e-12)


def test_trace_identity():
    """sum of all eigenvalues = int C(x, x) dx = 2a for the unit-amplitude 1-D kernel."""
    a, eta = 0.25, 0.2
    n = 4000
    lam, _, _, _ = kl.eig1d(a, eta, n)
    # tail beyond the last root: lambda_k ~ 2c / w_k^2 with w_k ~ k pi / (2a)
    tail = 8.0 * (1.0 / eta) * a * a / (np.pi ** 2 * n)
    assert abs(lam.sum() + tail - 2 * a) < 1e-6


def test_region_field_modes_and_amplitude():
    """2-D modes are products; sigma^2 scales the field by sigma (eq. covariance)."""
    p = problem("cfg0")
    reg = dict(p["regions"][0])
    modes, tx, ty = kl.region_modes(reg)
    assert [(m["a"], m["b"]) for m in modes] == [(0, 0), (0, 1)]
    for m in modes:
        assert m["lam"] == pytest.approx(reg["sigma2"] * tx[0][m["a"]] * ty[0][m["b"]], rel=1e-15)
    pts = np.array([[0.1, 0.2], [0.3, 0.9]])
    f1 = kl.region_field(reg, pts)
    reg2 = dict(reg, sigma2=4.0)
    assert np.allclose(kl.region_field(reg2, pts), 2.0 * f1, rtol=1e-14)


def test_covariance_reconstruction():
    """With many modes the truncated sum of lambda f f approaches sigma^2 exp(-...)."""
    reg = {"rect": [0.0, 0.5, 0.0, 1.0], "nterm": 400, "sigma2": 1.5, "eta": [0.2, 0.3], "mean_logk": 0.0}
    pts = np.array([[0.2, 0.4], [0.3, 0.55]])
    F = kl.region_field(reg, pts)
    c = F[:, 0] @ F[:, 1]
    exact = 1.5 * np.exp(-0.1 / 0.2 - 0.15 / 0.3)
    assert abs(c - exact) < 0.03 * exact
