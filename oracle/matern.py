"""Oracle: isotropic Matern covariance and its Nystrom KL basis, plain numpy/scipy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 5 (eq. matern): C(x, x') = 2^(1-nu) / Gamma(nu) (sqrt(2 nu) rho)^nu
K_nu(sqrt(2 nu) rho), rho = |x - x'|_2 / lambda_c, C(x, x) = 1.
Section 5 (Nystrom method): collocation of the covariance eigenproblem at
quadrature nodes x_q with weights w_q gives B = W^1/2 Sigma W^1/2 (Sigma_kq =
C(x_k, x_q)) with eigenpairs (theta_j, Psi*_j); the eigenfunction at any x is
the interpolation formula psi_j(x) = theta_j^-1 sum_q sqrt(w_q) Psi*_jq
C(x, x_q).  The KL basis of the truncated field (eq. truncatedKL) is then
sigma sqrt(theta_j) psi_j(x).

Quadrature: the Q x Q midpoint rule on the unit square, w_q = 1/Q^2.  The
same node set is what the library uses; everything else here (Bessel function,
eigensolver, extension) is computed independently of it: scipy.special.kv and
LAPACK's symmetric eigensolver through numpy.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def matern(rho, nu: float) -> np.ndarray:
    """eq. matern as a function of rho = |x - x'| / lambda_c (array or scalar)."""
    rho = np.asarray(rho, dtype=np.float64)
    x = math.sqrt(2.0 * nu) * rho
    out = np.ones_like(x)
    pos = x > 0
    xp = x[pos]
    out[pos] = 2.0 ** (1.0 - nu) / math.gamma(nu) * xp ** nu * special.kv(nu, xp)
    return out


def nodes(Q: int) -> np.ndarray:
    """Midpoint nodes of the unit square, node q = i + Q j at ((i+1/2)/Q, (j+1/2)/Q)."""
    c = (np.arange(Q) + 0.5) / Q
    X, Y = np.meshgrid(c, c, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def cell_centres(n: int) -> np.ndarray:
    """Centres of the n x n cells, cell p = i + n j at ((i+1/2)/n, (j+1/2)/n)."""
    return nodes(n)


def nystrom(Q: int, nu: float, lam: float):
    """Eigenpairs of B = W^1/2 Sigma W^1/2, descending: theta [Q^2], Psi* [Q^2][Q^2]
    (column j is the eigenvector of theta_j)."""
    x = nodes(Q)
    w = 1.0 / (Q * Q)
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    B = w * matern(d / lam, nu)
    theta, V = np.linalg.eigh(B)
    order = np.argsort(theta)[::-1]
    return theta[order], V[:, order]


def basis(Q: int, nu: float, lam: float, sigma2: float, s: int, pts: np.ndarray):
    """KL basis sigma sqrt(theta_j) psi_j(x) at the points pts [P][2] for j < s,
    by the Nystrom interpolation formula: returns (theta [s], basis [s][P])."""
    theta, V = nystrom(Q, nu, lam)
    x = nodes(Q)
    w = 1.0 / (Q * Q)
    d = np.sqrt(((pts[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    C = matern(d / lam, nu)                                   # [P][Q^2]
    psi = (C @ (math.sqrt(w) * V[:, :s])) / theta[:s]        # [P][s]
    return theta[:s], (math.sqrt(sigma2) * np.sqrt(theta[:s]) * psi).T


def hierarchy_basis(Q: int, nu: float, lam: float, sigma2: float, s: int, G: int):
    """Basis on the cell centres of every MG level 0..G (n_g = 2^(g+1)),
    level-major like the library's field: (theta [s], basis [s][M])."""
    pts = np.concatenate([cell_centres(2 << g) for g in range(G + 1)])
    return basis(Q, nu, lam, sigma2, s, pts)
