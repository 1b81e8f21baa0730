"""Pins of the oracle's Matern covariance and Nystrom KL basis (Section 5,
eq. matern and the Nystrom method) against closed forms and exact identities."""
import math

import numpy as np
import pytest

from oracle import matern as om


@pytest.mark.parametrize("rho", [1e-6, 0.01, 0.3, 1.0, 2.5, 7.0])
def test_half_integer_smoothness_closed_forms(rho):
    # Matern with nu = p + 1/2 is exp(-sqrt(2nu) rho) times a polynomial
    a = math.sqrt(3.0) * rho
    b = math.sqrt(5.0) * rho
    assert abs(om.matern(rho, 0.5) - math.exp(-rho)) < 1e-15
    assert abs(om.matern(rho, 1.5) - (1 + a) * math.exp(-a)) < 1e-14
    assert abs(om.matern(rho, 2.5) - (1 + b + b * b / 3) * math.exp(-b)) < 1e-14


@pytest.mark.parametrize("nu", [0.5, 1.0, 2.0])
def test_covariance_at_zero_and_monotone(nu):
    r = np.array([0.0, 1e-12, 1e-3, 0.1, 1.0, 3.0])
    c = om.matern(r, nu)
    assert c[0] == 1.0 and abs(c[1] - 1.0) < 1e-9
    assert np.all(np.diff(c) <= 0) and np.all(np.diff(c[1:]) < 0) and c[-1] > 0


def test_nu_one_against_bessel_series():
    # K_1 from its power series (Abramowitz-Stegun 9.6.11), small argument
    x = 0.2
    gamma_e = 0.5772156649015329
    k1 = 1 / x + math.log(x / 2) * sum((x / 2) ** (2 * k + 1) / (math.factorial(k) * math.factorial(k + 1))
                                       for k in range(20))
    h = [sum(1.0 / i for i in range(1, k + 1)) for k in range(22)]
    k1 -= 0.5 * sum((x / 2) ** (2 * k + 1) * (h[k] + h[k + 1] - 2 * gamma_e)
                    / (math.factorial(k) * math.factorial(k + 1)) for k in range(20))
    rho = x / math.sqrt(2.0)
    assert abs(om.matern(rho, 1.0) - x * k1) < 1e-14


@pytest.mark.parametrize("nu,lam", [(0.5, 0.3), (1.0, 0.1), (2.0, 0.5)])
def test_nystrom_trace_and_positivity(nu, lam):
    # sum of all eigenvalues = trace(B) = sum_q w_q C(x_q, x_q) = |D| = 1
    th, V = om.nystrom(12, nu, lam)
    assert abs(th.sum() - 1.0) < 1e-12
    assert th[0] > 0 and np.all(np.diff(th) <= 1e-15) and th[-1] > -1e-12
    assert np.allclose(V.T @ V, np.eye(V.shape[0]), atol=1e-12)


def test_interpolation_formula_reproduces_nodes():
    # at a node the Nystrom formula gives back the eigenvector: psi_j(x_q) =
    # Psi*_jq / sqrt(w_q), so the basis there is sigma sqrt(theta_j) Psi*_jq Q
    Q, nu, lam, s = 10, 1.0, 0.3, 15
    th, V = om.nystrom(Q, nu, lam)
    th_s, b = om.basis(Q, nu, lam, 2.0, s, om.nodes(Q))
    want = math.sqrt(2.0) * np.sqrt(th[:s])[:, None] * V[:, :s].T * Q
    assert np.allclose(th_s, th[:s]) and np.max(np.abs(b - want)) < 1e-12


def test_truncated_variance_and_convergence_in_q():
    # the pointwise variance of the truncated field, sum_j basis_j(x)^2, tends
    # to sigma^2 as s grows (Mercer), and the leading eigenvalues settle as
    # the quadrature is refined
    nu, lam = 2.0, 0.5
    th8, _ = om.nystrom(8, nu, lam)
    th16, _ = om.nystrom(16, nu, lam)
    assert np.max(np.abs(th8[:5] - th16[:5]) / th16[:5]) < 2e-2
    pts = np.array([[0.5, 0.5], [0.1, 0.9], [0.31, 0.27]])
    _, b = om.basis(16, nu, lam, 1.0, 60, pts)
    var = (b ** 2).sum(0)
    assert np.all(np.abs(var - 1.0) < 2e-2)


def test_hierarchy_layout():
    th, b = om.hierarchy_basis(6, 0.5, 0.3, 1.0, 4, 2)
    assert b.shape == (4, 4 + 16 + 64)
    # the first level-0 cell centre is (1/4, 1/4)
    _, b0 = om.basis(6, 0.5, 0.3, 1.0, 4, np.array([[0.25, 0.25]]))
    assert np.allclose(b[:, 0], b0[:, 0])
