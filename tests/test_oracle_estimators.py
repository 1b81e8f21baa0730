"""Pins of the oracle's estimators (Sections 2-3): the printed L = 2
expansion of the recycling estimator, the telescoping identity, the
no-recycling special case, and the shift-variance formula against numpy."""
import math

import numpy as np
import pytest

from oracle import estimators as est


def _random_F(rng, N, R):
    """F[k] of shape [R, N_k, k+1] with correlated levels."""
    L = len(N) - 1
    F = []
    for k in range(L + 1):
        base = rng.standard_normal((R, N[k], 1))
        F.append(base + 0.1 * np.cumsum(rng.standard_normal((R, N[k], k + 1)), axis=2))
    return F


def test_L2_expansion_matches_general_formula():
    """The fully expanded L = 2 MG-MLMC estimator of Section 2.2."""
    rng = np.random.default_rng(0)
    N = [9, 5, 3]
    F = _random_F(rng, N, 1)
    F0 = lambda k: F[k][0, :, 0]
    F1 = lambda k: F[k][0, :, 1]
    F2 = lambda k: F[k][0, :, 2]
    expanded = (
        (F0(0).sum() + F0(1).sum() + F0(2).sum()) / (N[0] + N[1] + N[2])
        + ((F1(1) - F0(1)).sum() + (F1(2) - F0(2)).sum()) / (N[1] + N[2])
        + (F2(2) - F1(2)).sum() / N[2]
    )
    q = est.mlmc_estimate(F, reuse=True)["q_bar"]
    assert abs(q - expanded) <= 1e-14 * max(1.0, abs(expanded))


def test_telescoping_identity():
    """All samples at finest level L: sum_l Upsilon_l,reuse = mean of F_L."""
    rng = np.random.default_rng(1)
    L, N, R = 4, 37, 3
    F = [np.zeros((R, 0, k + 1)) for k in range(L)] + [rng.standard_normal((R, N, L + 1))]
    ups = est.upsilon(F, reuse=True)
    for r in range(R):
        want = math.fsum(F[L][r, :, L]) / N
        assert abs(math.fsum(ups[:, r]) - want) <= 1e-14 * max(1.0, abs(want))


def test_no_reuse_uses_only_own_level():
    rng = np.random.default_rng(2)
    N = [8, 4, 2]
    F = _random_F(rng, N, 2)
    ups = est.upsilon(F, reuse=False)
    for r in range(2):
        for l in range(3):
            d = F[l][r, :, l] - (F[l][r, :, l - 1] if l else 0.0)
            assert abs(ups[l, r] - d.mean()) <= 1e-14


def test_shift_variance_is_numpy_unbiased_over_R():
    rng = np.random.default_rng(3)
    N, R = [6, 3, 2], 7
    F = _random_F(rng, N, R)
    for reuse in (False, True):
        out = est.mlmc_estimate(F, reuse)
        ups = out["upsilon"]
        qr = ups.sum(axis=0)
        assert np.allclose(out["q_shift"], qr, rtol=0, atol=1e-14)
        assert abs(out["q_bar"] - qr.mean()) <= 1e-14
        assert abs(out["var_q"] - qr.var(ddof=1) / R) <= 1e-14
        assert np.allclose(out["var_level"], ups.var(axis=1, ddof=1) / R, rtol=1e-13, atol=1e-16)
        assert np.allclose(out["upsilon_bar"], ups.mean(axis=1), rtol=0, atol=1e-14)


def test_single_replica_mlmc_variance():
    """R = 1 without recycling: V = sum_l s_l^2 / N_l (eq. vardecomp)."""
    rng = np.random.default_rng(4)
    N = [50, 20, 8]
    F = _random_F(rng, N, 1)
    out = est.mlmc_estimate(F, reuse=False)
    want = 0.0
    for l in range(3):
        d = F[l][0, :, l] - (F[l][0, :, l - 1] if l else 0.0)
        want += d.var(ddof=1) / N[l]
    assert abs(out["var_q"] - want) <= 1e-14
    assert np.isnan(est.mlmc_estimate(F, reuse=True)["var_q"])


def test_reuse_weights_count_recycled_samples():
    """With F_l constant c_l over all samples, every level estimator returns
    c_l - c_{l-1} whatever the sample counts (the weights sum to one)."""
    N = [7, 3, 1]
    c = [1.0, 1.5, 1.75]
    F = [np.broadcast_to(np.array(c[: k + 1]), (2, N[k], k + 1)).copy() for k in range(3)]
    ups = est.upsilon(F, reuse=True)
    assert np.allclose(ups[:, 0], [1.0, 0.5, 0.25], rtol=0, atol=1e-15)
