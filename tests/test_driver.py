"""Level-adaptive MG-MLQMC driver (Section 3.4, Algorithm 1): the control flow
on a synthetic sampler whose level values are known in closed form, so the
estimate, its bias and the doubling pattern can be checked without a GPU."""
import math

import numpy as np

from paper_1806_05619_amd.driver import mg_mlqmc, _alpha_fit


class SyntheticSampler:
    """F_tau(n, r) = 1 - 4^-tau (1 + c (u - 1/2)) with u the n-th point of a
    shifted 1-D rank-1 lattice sequence: E[F_tau - F_tau-1] decays like 4^-tau
    (alpha = 2), the limit is Q = 1 and shift-to-shift variance falls with N."""

    def __init__(self, R=8, c=0.5, seed=3):
        self.R, self.nq, self.c = R, 1, c
        self.shifts = np.random.default_rng(seed).random(R)
        self.calls = []

    def sample(self, level, n_begin, n_end):
        self.calls.append((level, n_begin, n_end))
        n = np.arange(n_begin, n_end)
        # van der Corput order of the 2^20-point rule, as a lattice sequence
        rev = np.array([int(f"{k:020b}"[::-1], 2) for k in n], dtype=np.float64) / 2.0**20
        out = np.zeros((self.R, 1, level + 1, 2))
        for r in range(self.R):
            u = (rev * 0.6180339887498949 * 2.0**20 % 1.0 + self.shifts[r]) % 1.0
            prev = 0.0
            for t in range(level + 1):
                F = 1.0 - 4.0**-t * (1.0 + self.c * (u - 0.5))
                d = F - prev
                out[r, 0, t] = (d.sum(), (d * d).sum())
                prev = F
        return out


def test_alpha_fit_recovers_rate():
    ub = np.array([1.0] + [3.0 * 4.0**-l for l in range(1, 6)])
    assert abs(_alpha_fit(ub) - 2.0) < 1e-12
    assert _alpha_fit(np.array([1.0, 1e-3])) == 0.5       # one difference: no fit


def test_reaches_tolerance_and_is_accurate():
    for eps in (1e-2, 1e-3, 1e-4):
        S = SyntheticSampler()
        r = mg_mlqmc(S, eps, max_level=12)
        assert r["converged"]
        assert r["var"] <= eps * eps / 2
        assert r["bias"] <= eps / math.sqrt(2)
        assert abs(r["q_bar"] - 1.0) <= 3 * eps, (eps, r["q_bar"])
        assert abs(r["alpha"] - 2.0) < 0.2
        # N_l only doubles from 1, and each call solves exactly the new points
        for l, n in enumerate(r["N"]):
            assert n == 0 or n & (n - 1) == 0
        seen = {}
        for l, a, b in S.calls:
            assert a == seen.get(l, 0) and b == max(1, 2 * a)
            seen[l] = b


def test_levels_grow_as_tolerance_shrinks():
    Ls = [mg_mlqmc(SyntheticSampler(), eps, max_level=14)["L"] for eps in (1e-2, 1e-3, 1e-4)]
    assert Ls[0] >= 2 and Ls == sorted(Ls) and Ls[2] > Ls[0]
    # bias |Ubar_L| / (4 - 1) <= eps / sqrt(2) with Ubar_L ~ 3/4 4^-L
    for eps, L in zip((1e-2, 1e-3, 1e-4), Ls):
        assert 0.75 * 4.0**-L / 3.0 <= eps / math.sqrt(2) * 1.05


def test_stops_when_levels_or_points_run_out():
    r = mg_mlqmc(SyntheticSampler(), 1e-6, max_level=3)
    assert not r["converged"] and r["L"] == 3
    r = mg_mlqmc(SyntheticSampler(), 1e-9, max_level=12, max_points=64)
    assert not r["converged"] and r["N"].max() <= 64


class FakeServer:
    """Stands in for mlmc_server: capacity 5 samples per batch, QoIs
    F_l(n, r) = (n + 1) * 10^-l + r (two QoIs: that and its double)."""

    nq = 2

    def __init__(self):
        self.reqs = {}

    def capacity(self, level):
        return 5

    def submit(self, level, n0, n1, r0, r1, sums=False):
        assert n1 - n0 <= 5 and r1 - r0 == 1 and sums
        tag = len(self.reqs)
        self.reqs[tag] = (level, n0, n1, r0)
        return tag

    def collect(self, tags):
        # the library forms a request's level sums on the device; here they
        # are formed exactly (math.fsum) from the closed-form QoIs
        import math
        out = []
        for t in tags:
            level, n0, n1, r = self.reqs[t]
            n = np.arange(n0, n1, dtype=np.float64)[:, None]
            F = (n + 1.0) * 10.0 ** -np.arange(level + 1)[None, :] + r
            Q = np.stack([F, 2.0 * F], axis=-1)            # [B][level+1][nq]
            d = np.diff(np.concatenate([np.zeros((Q.shape[0], 1, 2)), Q], axis=1), axis=1)
            sums = np.array([[[[math.fsum(d[:, l, q]), math.fsum(d[:, l, q] ** 2)]
                               for l in range(level + 1)] for q in range(2)]])
            out.append(dict(status=0, qoi=Q, sums=sums, not_converged=0, max_rel_residual=-1.0))
        return out


def test_server_sampler_splits_requests_and_adds_level_sums():
    from paper_1806_05619_amd.driver import ServerSampler
    srv = FakeServer()
    s = ServerSampler(srv, num_shifts=3, first_shift=4).sample(2, 3, 15)
    # 12 points per shift in requests of at most 5, shifts 4..6 of the table
    assert len(srv.reqs) == 3 * 3
    assert sorted({q[3] for q in srv.reqs.values()}) == [4, 5, 6]
    for r in range(3):
        for q in range(2):
            n = np.arange(3, 15, dtype=np.float64)
            F = np.stack([(n + 1.0) * 10.0 ** -l + (r + 4) for l in range(3)], axis=1) * (q + 1)
            d = np.diff(np.concatenate([np.zeros((12, 1)), F], axis=1), axis=1)
            assert np.allclose(s[r, q, :, 0], d.sum(axis=0), rtol=1e-14, atol=0)
            assert np.allclose(s[r, q, :, 1], (d * d).sum(axis=0), rtol=1e-14, atol=0)


def test_prop1_on_the_optimal_sample_numbers():
    """Sample numbers of eq. nopt2, N_l ~ h_l^((beta+gamma) lam/(lam+1)),
    make the new fraction of every level but the finest exactly
    1 - rho^(-(beta+gamma) lam/(lam+1)) (Proposition 1); the report fits
    gamma and beta back from costs and variances built with those rates."""
    from paper_1806_05619_amd.driver import prop1_reduction, recycling_report
    rho, beta, gamma, L = 2.0, 4.0, 2.0, 12
    for lam in (1.0, 0.5):
        x = (beta + gamma) * lam / (lam + 1.0)
        total = rho ** (-x * np.arange(L + 1)) * 1e9       # N_l with recycling
        new = total - np.append(total[1:], 0.0)              # N'_l
        cost = rho ** (gamma * np.arange(L + 1))
        var = rho ** (-beta * np.arange(L + 1)) / total      # estimator variance, MC rate
        rep = recycling_report(new, cost, var, rho=rho, lam=lam)
        want = prop1_reduction(beta, gamma, lam, rho)
        assert np.allclose(rep["new_fraction"][:-1], want, rtol=1e-12)
        assert rep["new_fraction"][-1] == 1.0
        assert abs(rep["gamma"] - gamma) < 1e-9 and abs(rep["beta"] - beta) < 1e-9
        assert abs(rep["predicted_fraction"] - want) < 1e-9
    # Monte Carlo, beta = 2, gamma = 2, rho = 2: 1 - 2^-2 of every level is new
    assert abs(prop1_reduction(2.0, 2.0, 1.0, 2.0) - 0.75) < 1e-15


class FlakySampler(SyntheticSampler):
    """Reports one unconverged sample on every call at level 2."""

    def __init__(self, strict):
        super().__init__()
        from paper_1806_05619_amd.driver import _ConvergenceLog
        self.log = _ConvergenceLog(strict)

    @property
    def not_converged(self):
        return self.log.not_converged

    def sample(self, level, n_begin, n_end):
        out = super().sample(level, n_begin, n_end)
        self.log.note(1 if level == 2 else 0, 3.5e-10, f"level {level}")
        return out


def test_unconverged_samples_are_counted_or_raised():
    from paper_1806_05619_amd.driver import NotConvergedError
    r = mg_mlqmc(FlakySampler(strict=False), 1e-3, max_level=12)
    assert r["not_converged"] == sum(1 for l, _, _ in r["history"] if l == 2) > 0
    try:
        mg_mlqmc(FlakySampler(strict=True), 1e-3, max_level=12)
    except NotConvergedError as e:
        assert "level 2" in str(e)
    else:
        raise AssertionError("strict sampler did not raise")


def test_bias_denominator_forms():
    """Default: the geometric tail |Ubar_L| / (rho^alpha - 1); 'plus' takes the
    printed rho^alpha + 1, which stops earlier (smaller bias estimate)."""
    a = mg_mlqmc(SyntheticSampler(), 1e-4, max_level=14)
    b = mg_mlqmc(SyntheticSampler(), 1e-4, max_level=14, bias_denominator="plus")
    assert b["L"] <= a["L"]
    ub = a["estimate"]["upsilon_bar"][0][a["L"]]
    assert abs(a["bias"] - abs(ub) / (2.0 ** a["alpha"] - 1.0)) <= 1e-15 * a["bias"]
    try:
        mg_mlqmc(SyntheticSampler(), 1e-3, max_level=4, bias_denominator="other")
    except ValueError:
        pass
    else:
        raise AssertionError("unknown denominator accepted")
