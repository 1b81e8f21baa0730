"""Multilevel (quasi-)Monte Carlo estimators, written out from their
definitions with plain loops and exactly rounded sums (``math.fsum``).

TEST INFRASTRUCTURE ONLY (part of the oracle).

Data model: ``F[k]`` is an array of shape ``[R, N_k, k+1]`` holding the QoI
``F_l(y^(n)_{k,r})`` for l = 0..k of the N_k samples of shift r whose finest
level is k (the FMG solve of such a sample yields all coarser levels too).
``F_{-1} = 0``.
"""
from __future__ import annotations

import math

import numpy as np


def _delta(Fk: np.ndarray, r: int, n: int, l: int) -> float:
    """F_l - F_{l-1} of one sample, with F_{-1} = 0."""
    return float(Fk[r, n, l]) - (float(Fk[r, n, l - 1]) if l > 0 else 0.0)


def upsilon(F, reuse: bool) -> np.ndarray:
    """Upsilon_{l,r}, shape [L+1][R].

    reuse=False: the per-shift level estimator of the MLQMC method,
    (1/N_l) sum_n (F_l - F_{l-1})(y_{l,r}^(n))  (Section 3.2, eq. MLMC per shift).
    reuse=True: eq. Upsilon-reuse, every sample whose finest level k >= l
    contributes, weight 1 / sum_{i>=l} N_i.
    """
    L = len(F) - 1
    R = F[0].shape[0]
    N = [F[k].shape[1] for k in range(L + 1)]
    ups = np.zeros((L + 1, R))
    for r in range(R):
        for l in range(L + 1):
            ks = range(l, L + 1) if reuse else [l]
            terms = []
            den = 0
            for k in ks:
                den += N[k]
                for n in range(N[k]):
                    terms.append(_delta(F[k], r, n, l))
            ups[l, r] = math.fsum(terms) / den if den > 0 else 0.0
    return ups


def shift_statistics(ups: np.ndarray) -> dict:
    """Statistics over the R shifts (R >= 2).

    Q_r = sum_l Upsilon_{l,r}; Qbar = mean over r (eq. MLQMC / MGMLQMC);
    V[Qbar] = sum_r (Q_r - Qbar)^2 / (R(R-1)) (eq. varovershifts /
    var_of_mgmlqmc); Upsilon_bar_l = mean over r (eq. Upsilon-reuse-bar);
    V_l = sum_r (Upsilon_{l,r} - Upsilon_bar_l)^2 / (R(R-1))
    (eq. sample_variances).
    """
    Lp1, R = ups.shape
    q_shift = np.array([math.fsum(ups[:, r]) for r in range(R)])
    q_bar = math.fsum(q_shift) / R
    var_q = math.fsum((q - q_bar) ** 2 for q in q_shift) / (R * (R - 1))
    ups_bar = np.array([math.fsum(ups[l]) / R for l in range(Lp1)])
    var_level = np.array([math.fsum((ups[l, r] - ups_bar[l]) ** 2 for r in range(R))
                          / (R * (R - 1)) for l in range(Lp1)])
    return dict(q_shift=q_shift, q_bar=q_bar, var_q=var_q, upsilon_bar=ups_bar,
                var_level=var_level)


def mlmc_estimate(F, reuse: bool) -> dict:
    """Estimator outputs for one QoI.

    R >= 2: shift statistics of Upsilon (with or without recycling).
    R == 1, reuse=False: plain MLMC (eq. MLMC) with the variance of
    eq. vardecomp, V = sum_l s_l^2 / N_l, s_l^2 the unbiased sample variance of
    F_l - F_{l-1}.  R == 1 with reuse has no valid variance estimate
    (eq. vardecomp2 has unknown covariances): variances are NaN.
    """
    ups = upsilon(F, reuse)
    R = ups.shape[1]
    if R >= 2:
        out = shift_statistics(ups)
    else:
        L = len(F) - 1
        q = math.fsum(ups[:, 0])
        if reuse:
            var_level = np.full(L + 1, np.nan)
        else:
            var_level = np.empty(L + 1)
            for l in range(L + 1):
                N = F[l].shape[1]
                d = [_delta(F[l], 0, n, l) for n in range(N)]
                m = math.fsum(d) / N
                var_level[l] = (math.fsum((v - m) ** 2 for v in d) / (N - 1)) / N \
                    if N > 1 else np.nan
        out = dict(q_shift=np.array([q]), q_bar=q,
                   var_q=float(math.fsum(var_level)) if not reuse else float("nan"),
                   upsilon_bar=ups[:, 0].copy(), var_level=var_level)
    out["upsilon"] = ups
    return out
