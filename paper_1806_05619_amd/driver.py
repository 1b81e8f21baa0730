"""Level-adaptive MG-MLQMC driver (Section 3.4, Algorithm 1).

The driver decides how many lattice points each level gets; the samples
themselves are solved by the library (`SampleAndSolve` of the algorithm is one
`mlmc_fmg_solve` call over a new range of lattice points for all R shifts,
which also yields the recycled coarse solutions), and the estimators come from
`mlmc_estimate`.

Algorithm (Section 3.4): start with L = -1; while L < 2 or the bias estimate
exceeds eps / sqrt(2), add a level; while the variance estimate (eq.
var_of_mgmlqmc) exceeds eps^2 / 2, double N_l (N_l = max(1, 2 N_l)) on the
level l <= L with the largest V_l / C_l (eq. sample_variances over the
measured cost per sample C_l) and solve the new points.  The bias estimate is
|Upsilon-bar_L| / (rho^alpha - 1) with alpha from a least-squares fit of
log2 |Upsilon-bar_l| over l = 1..L; the paper prints rho^alpha + 1 in eq. bias,
while the geometric tail sum_{j>=1} rho^(-alpha j) that the estimate stands for
(and the MLMC literature it cites) gives rho^alpha - 1.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import mlmc_estimate


class GpuSampler:
    """SampleAndSolve on the GPU: lattice points [n_begin, n_end) of every shift
    on finest level `level`, returning the level-difference sums
    [R][nq][level+1][2] on the host."""

    def __init__(self, ctx):
        import torch
        self.ctx = ctx
        self.R = ctx.num_shifts
        self.nq = ctx.nq
        self._torch = torch

    def sample(self, level, n_begin, n_end):
        torch = self._torch
        s = torch.zeros((self.R, self.nq, level + 1, 2), dtype=torch.float64,
                        device=torch.device("cuda", self.ctx.device))
        self.ctx.fmg_solve(self.ctx.lattice(level, n_begin, n_end, 0, self.R), sums=s)
        return s.cpu().numpy()          # synchronising copy: the timer sees the solve


class GpuMcSampler:
    """SampleAndSolve with Monte Carlo points (plain MLMC, Section 2): R
    independent replicas of i.i.d. standard normal vectors play the role of
    the R random shifts, so the same estimators (eq. MLQMC, eq. varovershifts
    and their recycling forms) apply.  normals(level, replica, n_begin, n_end)
    returns the [n_end - n_begin][s] normals of that replica, drawn once per
    (level, replica) stream; each replica is one explicit-points solve."""

    def __init__(self, ctx, normals, num_replicas):
        import torch
        self.ctx = ctx
        self.R = int(num_replicas)
        self.nq = ctx.nq
        self.normals = normals
        self._torch = torch

    def sample(self, level, n_begin, n_end):
        torch = self._torch
        dev = torch.device("cuda", self.ctx.device)
        out = torch.zeros((self.R, self.nq, level + 1, 2), dtype=torch.float64, device=dev)
        for r in range(self.R):
            y = torch.as_tensor(self.normals(level, r, n_begin, n_end), dtype=torch.float64)
            self.ctx.fmg_solve(self.ctx.explicit(level, y.to(dev).contiguous()), sums=out[r:r + 1])
        return out.cpu().numpy()


class ServerSampler:
    """SampleAndSolve through the serving loop (mlmc_server): the new lattice
    points of every shift become requests (split to the server's capacity at
    the level), which the server batches with whatever else is queued; the
    level-difference sums are formed on the host from the returned QoIs."""

    def __init__(self, server, num_shifts, first_shift=0):
        self.srv = server
        self.R = int(num_shifts)
        self.r0 = int(first_shift)      # shifts r0 .. r0+R-1 of the server's table
        self.nq = server.nq

    def sample(self, level, n_begin, n_end):
        cap = self.srv.capacity(level)
        reqs = [(level, a, min(a + cap, n_end), self.r0 + r, self.r0 + r + 1)
                for r in range(self.R) for a in range(n_begin, n_end, cap)]
        tags = [self.srv.submit(*q) for q in reqs]
        sums = np.zeros((self.R, self.nq, level + 1, 2))
        for q, res in zip(reqs, self.srv.collect(tags)):
            if res["status"] != 0:
                raise RuntimeError(f"request {q} failed with status {res['status']}")
            F = res["qoi"]                                   # [B][level+1][nq]
            d = F.copy()
            d[:, 1:, :] -= F[:, :-1, :]                      # F_l - F_(l-1), F_(-1) = 0
            r = q[3] - self.r0
            sums[r, :, :, 0] += d.sum(axis=0).T
            sums[r, :, :, 1] += (d * d).sum(axis=0).T
        return sums


def _alpha_fit(ubar):
    """Least-squares slope of -log2 |Upsilon-bar_l| over l = 1..L (at least 0.5)."""
    lv = np.arange(1, len(ubar))
    y = np.log2(np.maximum(np.abs(ubar[1:]), 1e-300))
    if len(lv) < 2:
        return 0.5
    slope = np.polyfit(lv, y, 1)[0]
    return max(-slope, 0.5)


def mg_mlqmc(sampler, eps, max_level, qoi=0, rho=2.0, reuse=True, max_points=None,
             clock=time.perf_counter):
    """Run Algorithm 1 to tolerance eps (root mean square error) on levels
    0..max_level.  Returns the estimate, its variance and bias estimates, the
    points per level, the measured cost per sample and the call history."""
    R, nq = sampler.R, sampler.nq
    L1 = max_level + 1
    N = np.zeros(L1, dtype=np.int64)
    N_old = np.zeros(L1, dtype=np.int64)
    sums = np.zeros((L1, R, nq, L1, 2))
    V = np.full(L1, np.inf)
    C = np.zeros(L1)
    solved = np.zeros(L1, dtype=np.int64)      # samples timed per level
    history = []
    est = None

    def sample_and_solve(l):
        nonlocal est
        t0 = clock()
        s = sampler.sample(l, int(N_old[l]), int(N[l]))
        dt = clock() - t0
        sums[l, :, :, : l + 1, :] += s
        new = int(N[l] - N_old[l]) * R
        C[l] = (C[l] * solved[l] + dt) / (solved[l] + new)     # mean time per sample
        solved[l] += new
        history.append((l, int(N_old[l]), int(N[l])))
        est = mlmc_estimate(N, sums, R, nq, reuse)
        V[: l + 1] = est["var_level"][qoi][: l + 1]
        N_old[l] = N[l]

    def bias(L):
        ub = est["upsilon_bar"][qoi][: L + 1]
        a = _alpha_fit(ub)
        return abs(ub[L]) / (rho ** a - 1.0), a

    L, converged, alpha, b = -1, True, float("nan"), float("inf")
    while True:
        if L >= 2:
            b, alpha = bias(L)
            if b <= eps / math.sqrt(2.0):
                break
        if L + 1 > max_level:
            converged = False
            break
        L += 1
        while np.sum(V[: L + 1]) > eps * eps / 2.0:
            ratio = np.where(C[: L + 1] > 0, V[: L + 1] / np.where(C[: L + 1] > 0, C[: L + 1], 1.0),
                             np.inf)
            l = int(np.argmax(ratio))
            n_new = max(1, 2 * int(N[l]))
            if max_points is not None and n_new > max_points:
                converged = False
                break
            N[l] = n_new
            sample_and_solve(l)
        if not converged:
            break
    return dict(q_bar=float(est["q_bar"][qoi]), var=float(np.sum(V[: L + 1])), bias=b,
                alpha=alpha, L=L, N=N[: L + 1].copy(), cost=C[: L + 1].copy(),
                converged=converged, history=history, estimate=est)


def _rate(values, rho):
    """Least-squares slope of log_rho |values_l| over l = 1..L (None if < 2 levels)."""
    v = np.abs(np.asarray(values, dtype=np.float64))
    lv = np.arange(1, len(v))
    if len(lv) < 2 or np.any(v[1:] <= 0):
        return None
    return float(np.polyfit(lv, np.log(v[1:]) / np.log(rho), 1)[0])


def prop1_reduction(beta, gamma, lam=1.0, rho=2.0):
    """Proposition 1: with geometric refinement h_l = rho h_(l+1) and the
    sample numbers of eq. nopt2, recycling leaves a fraction
    1 - rho^(-(beta+gamma) lam/(lam+1)) of the samples of every level
    (but the finest) to be computed; lam = 1 for Monte Carlo."""
    return 1.0 - rho ** (-(beta + gamma) * lam / (lam + 1.0))


def recycling_report(N, cost, var=None, rho=2.0, lam=1.0):
    """Recycled fractions of a run (Section 3.3, Proposition 1).  N[l]:
    samples whose finest level is l (the new ones, N'_l); the samples
    available on level l are sum_(k >= l) N[k].  Returns the new fraction
    N'_l / N_l per level, the cost ratio with and without recycling for the
    measured cost per sample, the cost rate gamma fitted to `cost`, and, if
    per-level variances `var` of the level estimators are given, beta fitted
    to var[l] * N_l (the per-sample variance under a Monte Carlo rate) and
    Proposition 1's prediction for those rates."""
    N = np.asarray(N, dtype=np.float64)
    cost = np.asarray(cost, dtype=np.float64)
    total = np.cumsum(N[::-1])[::-1]
    frac = np.where(total > 0, N / np.where(total > 0, total, 1.0), np.nan)
    out = dict(new_fraction=frac.tolist(), available=total.tolist(),
               cost_ratio=float(np.sum(N * cost) / np.sum(total * cost)))
    gamma = _rate(cost, rho)
    out["gamma"] = gamma
    if var is not None:
        v = np.asarray(var, dtype=np.float64) * total
        b = _rate(v, rho)
        out["beta"] = None if b is None else -b
        if b is not None and gamma is not None:
            out["predicted_fraction"] = prop1_reduction(-b, gamma, lam, rho)
    return out
