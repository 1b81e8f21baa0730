"""Pins of the oracle's truncated KL expansion (Section 5) for the separable
exponential covariance: eigen-equation residual by quadrature,
orthonormality, the trace identity of Section 6, Mercer convergence of the
covariance, and structural facts about the 2-D mode ordering."""
import math

import numpy as np
import pytest
from scipy import integrate

LAMS = [0.3, 0.1, 0.05]


def _char(lam, w):
    return (lam * lam * w * w - 1.0) * math.sin(w) - 2.0 * lam * w * math.cos(w)


@pytest.mark.parametrize("lam", LAMS)
def test_one_root_per_interval(oracle_mod, lam):
    for k in range(1, 41):
        lo, hi = (k - 1) * math.pi, k * math.pi
        ws = np.linspace(lo, hi, 4001)[1:-1]
        sg = np.sign([_char(lam, w) for w in ws])
        assert np.count_nonzero(np.diff(sg)) == 1, k
        w = oracle_mod.kl_root(lam, k)
        assert lo < w < hi
        # the characteristic function changes sign within 1e-15 relative of w
        d = 1e-15 * w
        assert _char(lam, w - d) * _char(lam, w + d) <= 0.0


@pytest.mark.parametrize("lam", LAMS)
@pytest.mark.parametrize("k", [1, 2, 5, 17])
def test_eigen_equation_residual(oracle_mod, lam, k):
    """int_0^1 exp(-|x-t|/lam) psi_k(t) dt = theta_k psi_k(x)."""
    w = oracle_mod.kl_root(lam, k)
    th = oracle_mod.kl_theta(lam, w)
    for x in [0.0, 0.13, 0.5, 0.77, 1.0]:
        f = lambda t: math.exp(-abs(x - t) / lam) * oracle_mod.kl_psi(lam, w, t)
        left = integrate.quad(f, 0.0, x, epsabs=1e-15, epsrel=1e-14, limit=400)[0] if x > 0 else 0.0
        right = integrate.quad(f, x, 1.0, epsabs=1e-15, epsrel=1e-14, limit=400)[0] if x < 1 else 0.0
        assert abs(left + right - th * oracle_mod.kl_psi(lam, w, x)) <= 1e-12


@pytest.mark.parametrize("lam", LAMS)
def test_orthonormal(oracle_mod, lam):
    xg, wg = np.polynomial.legendre.leggauss(400)
    xg, wg = 0.5 * (xg + 1), 0.5 * wg
    K = 12
    ws = [oracle_mod.kl_root(lam, k) for k in range(1, K + 1)]
    Psi = np.array([[oracle_mod.kl_psi(lam, w, x) for x in xg] for w in ws])
    G = (Psi * wg) @ Psi.T
    assert np.max(np.abs(G - np.eye(K))) <= 1e-12


@pytest.mark.parametrize("lam", [0.3, 0.1])
def test_trace_identity(oracle_mod, lam):
    """sum_j theta_j = |D| = 1 (Section 6), in 1-D and hence for the 2-D products."""
    p = 3000
    th = np.array([oracle_mod.kl_theta(lam, oracle_mod.kl_root(lam, k)) for k in range(1, p + 1)])
    tail = 2.0 / (lam * math.pi**2 * (p - 1))      # > sum_{k>p} 2 lam / (1 + lam^2 w_k^2)
    assert 1.0 - tail < th.sum() < 1.0
    assert np.all(np.diff(th) < 0)


def test_mercer_covariance(oracle_mod):
    """sum_k theta_k psi_k(x) psi_k(x') -> exp(-|x-x'|/lam) away from the diagonal."""
    lam, p = 0.3, 1500
    ws = [oracle_mod.kl_root(lam, k) for k in range(1, p + 1)]
    for x, xp in [(0.1, 0.4), (0.5, 0.9), (0.0, 1.0), (0.25, 0.3)]:
        c = sum(oracle_mod.kl_theta(lam, w) * oracle_mod.kl_psi(lam, w, x) * oracle_mod.kl_psi(lam, w, xp)
                for w in ws)
        assert abs(c - math.exp(-abs(x - xp) / lam)) < 2e-3


def test_first_eigenvalues_lambda_03(oracle_mod):
    # eigenvalues from an independent bisection on the characteristic equation
    th = [oracle_mod.kl_theta(0.3, oracle_mod.kl_root(0.3, k)) for k in (1, 2)]
    assert abs(th[0] - 0.436249) < 1e-6 and abs(th[1] - 0.216812) < 1e-6


@pytest.mark.parametrize("lam,s", [(0.3, 10), (0.3, 100), (0.1, 400), (0.05, 1000)])
def test_mode_table_structure(oracle_mod, lam, s):
    mi, mj, th = oracle_mod.kl_modes(lam, s)
    assert np.all(np.diff(th) <= 0)
    kept = set(zip(mi.tolist(), mj.tolist()))
    assert len(kept) == s
    # the exact top-s set is closed under lowering either index
    for i, j in kept:
        if i > 1:
            assert (i - 1, j) in kept
        if j > 1:
            assert (i, j - 1) in kept
    # ties theta_i theta_j == theta_j theta_i: keep the smaller i first
    for m in range(s - 1):
        if th[m] == th[m + 1]:
            assert mi[m] < mi[m + 1]
    # a pair split by the cut keeps (i, j) with i < j
    for i, j in kept:
        if i != j and (j, i) not in kept:
            assert i < j
    # every product is the product of the 1-D eigenvalues
    for m in range(0, s, max(1, s // 20)):
        ti = oracle_mod.kl_theta(lam, oracle_mod.kl_root(lam, int(mi[m])))
        tj = oracle_mod.kl_theta(lam, oracle_mod.kl_root(lam, int(mj[m])))
        assert th[m] == ti * tj


def test_field_is_kl_sum(oracle_mod):
    """z is linear in y; unit vectors give the scaled product eigenfunctions;
    sigma^2 = 0 gives z = 0 exactly (a = 1)."""
    P = oracle_mod.Problem(4, 3, 10, 0.3, 2.0)
    k = 1
    mi, mj, th = oracle_mod.kl_modes(0.3, 10)
    rng = np.random.default_rng(3)
    y1, y2 = rng.standard_normal(10), rng.standard_normal(10)
    z1, z2, z12 = P.field(y1, k), P.field(y2, k), P.field(2.0 * y1 - y2, k)
    assert np.max(np.abs(z12 - (2 * z1 - z2))) < 1e-13
    for m in (0, 3, 9):
        e = np.zeros(10)
        e[m] = 1.0
        z = P.field(e, k)
        for g, n, sl in P.level_slices(k):
            c = (np.arange(n) + 0.5) / n
            wi = oracle_mod.kl_root(0.3, int(mi[m]))
            wj = oracle_mod.kl_root(0.3, int(mj[m]))
            ref = math.sqrt(2.0) * math.sqrt(th[m]) * np.outer(
                [oracle_mod.kl_psi(0.3, wj, x) for x in c], [oracle_mod.kl_psi(0.3, wi, x) for x in c])
            assert np.max(np.abs(z[sl].reshape(n, n) - ref)) < 1e-14
    P0 = oracle_mod.Problem(4, 3, 10, 0.3, 0.0)
    assert np.all(P0.field(y1, 2) == 0.0)


def test_field_pointwise_variance(oracle_mod):
    """Var z(x) = sigma^2 sum_{m<=s} theta_m psi_m(x)^2 <= sigma^2, increasing in s."""
    lam = 0.3
    prev = None
    for s in (10, 40, 100):
        P = oracle_mod.Problem(4, 1, s, lam, 1.0)
        Z = np.array([P.field(np.eye(s)[m], 0) for m in range(s)])   # rows: basis functions
        var = (Z**2).sum(axis=0)
        assert np.all(var <= 1.0 + 1e-12)
        if prev is not None:
            assert np.all(var >= prev - 1e-15)
        prev = var
