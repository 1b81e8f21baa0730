"""Level-adaptive MG-MLQMC driver (Section 3.4).

The driver decides how many lattice points each level gets; the samples
themselves are solved by the library (one sampling call is one
`mlmc_fmg_solve` over a new range of lattice points for all R shifts, which
also yields the recycled coarse solutions, or the equivalent requests to the
serving loop), and the estimators come from `mlmc_estimate`.

The run is steered by the two halves of the mean square error: the
statistical error, the variance estimate of eq. var_of_mgmlqmc built from
the per-level shift variances of eq. sample_variances, must fall below
eps^2 / 2, and the bias, estimated from the last level difference Upsilon-bar_L
of eq. Upsilon-reuse-bar, must fall below eps / sqrt(2) (eq. bias).  While the
variance is too large, the level with the most variance per unit of measured
cost per sample gets twice its lattice points (a lattice sequence keeps its
earlier points, so only the new ones are solved); once it is small enough, a
level is added if the bias is too large.  The bias estimate assumes the level
differences decay geometrically, |Upsilon-bar_l| ~ rho^(-alpha l), with alpha
fitted over l = 1..L: the neglected tail sum_{j>=1} rho^(-alpha j)
|Upsilon-bar_L| is |Upsilon-bar_L| / (rho^alpha - 1).  The paper prints
rho^alpha + 1 in that denominator; `bias_denominator="plus"` selects the
printed form.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import MLMC_E_NOCONV, mlmc_estimate


class NotConvergedError(RuntimeError):
    """A sampling call returned samples whose refinement stopped above rtol."""


class _ConvergenceLog:
    """Unconverged samples seen by a sampler: counted, or raised at once."""

    def __init__(self, strict):
        self.strict = bool(strict)
        self.not_converged = 0
        self.max_rel_residual = -1.0

    def note(self, count, max_rel_residual, what):
        self.max_rel_residual = max(self.max_rel_residual, float(max_rel_residual))
        if count:
            self.not_converged += int(count)
            if self.strict:
                raise NotConvergedError(f"{count} sample(s) of {what} stopped above rtol "
                                        f"(largest final residual ratio {max_rel_residual:.3e})")


class GpuSampler(_ConvergenceLog):
    """One sampling call on the GPU: lattice points [n_begin, n_end) of every
    shift on finest level `level`, returning the level-difference sums
    [R][nq][level+1][2] on the host.  Samples whose refinement stopped above
    rtol are counted in `not_converged` (strict=True raises instead)."""

    def __init__(self, ctx, strict=False):
        import torch
        super().__init__(strict)
        self.ctx = ctx
        self.R = ctx.num_shifts
        self.nq = ctx.nq
        self._torch = torch

    def sample(self, level, n_begin, n_end):
        torch = self._torch
        s = torch.zeros((self.R, self.nq, level + 1, 2), dtype=torch.float64,
                        device=torch.device("cuda", self.ctx.device))
        info = self.ctx.fmg_solve(self.ctx.lattice(level, n_begin, n_end, 0, self.R), sums=s,
                                  want_info=True)
        self.note(info["not_converged"], info["max_rel_residual"],
                  f"level {level}, points {n_begin}..{n_end}")
        return s.cpu().numpy()


class GpuMcSampler(_ConvergenceLog):
    """One sampling call with Monte Carlo points (plain MLMC, Section 2): R
    independent replicas of i.i.d. standard normal vectors play the role of
    the R random shifts, so the same estimators (eq. MLQMC, eq. varovershifts
    and their recycling forms) apply.  normals(level, replica, n_begin, n_end)
    returns the [n_end - n_begin][s] normals of that replica, drawn once per
    (level, replica) stream; each replica is one explicit-points solve."""

    def __init__(self, ctx, normals, num_replicas, strict=False):
        import torch
        super().__init__(strict)
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
            info = self.ctx.fmg_solve(self.ctx.explicit(level, y.to(dev).contiguous()),
                                      sums=out[r:r + 1], want_info=True)
            self.note(info["not_converged"], info["max_rel_residual"],
                      f"level {level}, replica {r}")
        return out.cpu().numpy()


class ServerSampler(_ConvergenceLog):
    """One sampling call through the serving loop (mlmc_server): the new
    lattice points of every shift become requests (split to the server's
    capacity at the level), which the server batches with whatever else is
    queued.  The server forms each request's level-difference sums on the
    device; this sampler only adds up the sums of a shift's requests."""

    def __init__(self, server, num_shifts, first_shift=0, strict=False):
        super().__init__(strict)
        self.srv = server
        self.R = int(num_shifts)
        self.r0 = int(first_shift)      # shifts r0 .. r0+R-1 of the server's table
        self.nq = server.nq

    def sample(self, level, n_begin, n_end):
        cap = self.srv.capacity(level)
        reqs = [(level, a, min(a + cap, n_end), self.r0 + r, self.r0 + r + 1)
                for r in range(self.R) for a in range(n_begin, n_end, cap)]
        tags = [self.srv.submit(*q, sums=True) for q in reqs]
        sums = np.zeros((self.R, self.nq, level + 1, 2))
        for q, res in zip(reqs, self.srv.collect(tags)):
            if res["status"] not in (0, MLMC_E_NOCONV):
                raise RuntimeError(f"request {q} failed with status {res['status']}")
            self.note(res.get("not_converged", 0), res.get("max_rel_residual", -1.0),
                      f"request {q}")
            sums[q[3] - self.r0] += res["sums"][0]
        return sums


def _alpha_fit(ubar):
    """Least-squares slope of -log2 |Upsilon-bar_l| over l = 1..L (at least 0.5)."""
    lv = np.arange(1, len(ubar))
    y = np.log2(np.maximum(np.abs(ubar[1:]), 1e-300))
    if len(lv) < 2:
        return 0.5
    slope = np.polyfit(lv, y, 1)[0]
    return max(-slope, 0.5)


class AdaptiveEstimator:
    """State of an adaptive MG-MLQMC run on levels 0..max_level: the summed
    level differences per origin level, the lattice points per level, the
    measured cost per sample and the current estimate."""

    def __init__(self, sampler, max_level, qoi=0, rho=2.0, reuse=True, max_points=None,
                 bias_denominator="minus", clock=time.perf_counter):
        if bias_denominator not in ("minus", "plus"):
            raise ValueError("bias_denominator is 'minus' (rho^alpha - 1) or 'plus' (as printed)")
        self.sampler, self.qoi, self.rho, self.reuse = sampler, int(qoi), float(rho), bool(reuse)
        self.max_points, self.clock = max_points, clock
        self.sign = -1.0 if bias_denominator == "minus" else 1.0
        L1 = int(max_level) + 1
        R, nq = sampler.R, sampler.nq
        self.points = np.zeros(L1, dtype=np.int64)        # lattice points per origin level
        self.sums = np.zeros((L1, R, nq, L1, 2))
        self.cost = np.zeros(L1)                          # mean seconds per sample
        self.timed = np.zeros(L1, dtype=np.int64)
        self.var = np.full(L1, np.inf)                    # per-level estimator variance
        self.history = []
        self.est = None
        self.L = -1

    def grow(self, l, n_new):
        """Solve lattice points [points[l], n_new) of every shift at level l."""
        n_old = int(self.points[l])
        t0 = self.clock()
        s = self.sampler.sample(l, n_old, n_new)
        dt = self.clock() - t0
        self.sums[l, :, :, : l + 1, :] += s
        added = (n_new - n_old) * self.sampler.R
        self.cost[l] = (self.cost[l] * self.timed[l] + dt) / (self.timed[l] + added)
        self.timed[l] += added
        self.points[l] = n_new
        self.history.append((l, n_old, n_new))
        self.est = mlmc_estimate(self.points, self.sums, self.sampler.R, self.sampler.nq,
                                 self.reuse)
        self.var[: l + 1] = self.est["var_level"][self.qoi][: l + 1]

    def variance(self):
        return float(np.sum(self.var[: self.L + 1]))

    def bias(self):
        """(bias estimate, fitted alpha) from the level differences 0..L."""
        ub = self.est["upsilon_bar"][self.qoi][: self.L + 1]
        alpha = _alpha_fit(ub)
        return abs(ub[self.L]) / (self.rho ** alpha + self.sign), alpha

    def best_level(self):
        """The level with the most variance per unit of cost (unsolved first)."""
        v, c = self.var[: self.L + 1], self.cost[: self.L + 1]
        gain = np.where(c > 0, v / np.where(c > 0, c, 1.0), np.inf)
        return int(np.argmax(gain))

    def reduce_variance(self, eps):
        """Double the points of the best level until the variance meets
        eps^2 / 2; False if the point budget runs out first."""
        while self.variance() > eps * eps / 2.0:
            l = self.best_level()
            n_new = max(1, 2 * int(self.points[l]))
            if self.max_points is not None and n_new > self.max_points:
                return False
            self.grow(l, n_new)
        return True

    def run(self, eps):
        """Levels are added until the bias meets eps / sqrt(2) (at least three
        levels, so that alpha can be fitted), the variance being reduced to
        eps^2 / 2 on every level set."""
        converged, bias, alpha = True, float("inf"), float("nan")
        while True:
            if self.L >= 2:
                bias, alpha = self.bias()
                if bias <= eps / math.sqrt(2.0):
                    break
            if self.L + 1 >= len(self.points):
                converged = False
                break
            self.L += 1
            if not self.reduce_variance(eps):
                converged = False
                break
        L = self.L
        return dict(q_bar=float(self.est["q_bar"][self.qoi]), var=self.variance(), bias=bias,
                    alpha=alpha, L=L, N=self.points[: L + 1].copy(),
                    cost=self.cost[: L + 1].copy(), converged=converged,
                    history=list(self.history), estimate=self.est,
                    not_converged=int(getattr(self.sampler, "not_converged", 0)))


def mg_mlqmc(sampler, eps, max_level, qoi=0, rho=2.0, reuse=True, max_points=None,
             bias_denominator="minus", clock=time.perf_counter):
    """Adaptive MG-MLQMC (reuse=True) or MLQMC (reuse=False) to root mean
    square error eps on levels 0..max_level (Section 3.4).  Returns the
    estimate, its variance and bias estimates, the points per level, the
    measured cost per sample, the sampling history and the count of samples
    whose refinement stopped above rtol."""
    return AdaptiveEstimator(sampler, max_level, qoi=qoi, rho=rho, reuse=reuse,
                             max_points=max_points, bias_denominator=bias_denominator,
                             clock=clock).run(eps)


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
