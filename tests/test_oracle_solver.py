"""Pins of the oracle's discretisation, direct solve and full multigrid
(Sections 4 and 6): spectral solve for a = 1, the constant-coefficient series
solution, O(h^2) convergence on a manufactured solution, the FMG figure's visit
sequence, FMG agreeing with the direct solve, and discretisation accuracy of
the fixed-cycle FMG."""
import math

import numpy as np
import pytest
from scipy import fft

import synth


def series_values():
    """mean of u and u(1/2,1/2) for -Lap u = 1 on the unit square, u = 0 on
    the boundary, from the classical Fourier series (x(1-x)/2 minus a
    cosh-series correction)."""
    mean = 1.0 / 12.0 - math.fsum(16.0 * math.tanh(m * math.pi / 2) / (math.pi**5 * m**5)
                                  for m in range(1, 40001, 2))
    ctr = 1.0 / 8.0 - math.fsum(4.0 * (-1) ** ((m - 1) // 2) / (math.pi**3 * m**3 * math.cosh(m * math.pi / 2))
                                for m in range(1, 401, 2))
    return mean, ctr


def test_series_values_recomputed():
    # 30-digit values of the same series (mpmath nsum), stored with the tests
    mean, ctr = series_values()
    assert abs(mean - 0.0351442537387884289) < 1e-16
    assert abs(ctr - 0.0736713532815138156) < 1e-16


@pytest.mark.parametrize("n", [2, 4, 8, 32])
def test_direct_solve_matches_dst(oracle_mod, n):
    """a = 1: the cell-centred operator with odd wall reflection is
    diagonalised by the DST-II basis, eigenvalues 4 sin^2(k pi / 2n) / h^2."""
    rng = np.random.default_rng(n)
    f = rng.standard_normal((n, n))
    lam1 = 4.0 * np.sin(np.arange(1, n + 1) * np.pi / (2 * n)) ** 2 * n * n
    fh = fft.dstn(f, type=2)
    u_ref = fft.idstn(fh / (lam1[:, None] + lam1[None, :]), type=2)
    u = oracle_mod.direct_solve(n, np.ones(n * n), f.reshape(-1)).reshape(n, n)
    assert np.max(np.abs(u - u_ref)) <= 1e-13 * max(1.0, np.max(np.abs(u_ref)))


def test_constant_coefficient_convergence(oracle_mod):
    mean, ctr = series_values()
    errs = []
    for n in (16, 32, 64, 128):
        u = oracle_mod.direct_solve(n, np.ones(n * n), np.ones(n * n))
        qm, qc = oracle_mod.qoi(n, u)
        errs.append((qm - mean, qc - ctr))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(np.abs(ratios - 4.0) < 0.1), ratios
    assert np.all(np.abs(errs[-1]) < 1e-5)


def _manufactured(n):
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c, indexing="xy")      # X varies along i (fastest)
    pi = math.pi
    a = np.exp(0.5 * np.sin(2 * pi * X) * np.cos(2 * pi * Y))
    u = np.sin(pi * X) * np.sin(pi * Y)
    ax = a * pi * np.cos(2 * pi * X) * np.cos(2 * pi * Y)
    ay = -a * pi * np.sin(2 * pi * X) * np.sin(2 * pi * Y)
    ux = pi * np.cos(pi * X) * np.sin(pi * Y)
    uy = pi * np.sin(pi * X) * np.cos(pi * Y)
    f = -(ax * ux + ay * uy - 2 * pi * pi * a * u)
    return a, u, f


def test_manufactured_solution_second_order(oracle_mod):
    errs = []
    for n in (16, 32, 64, 128):
        a, u_ex, f = _manufactured(n)
        u = oracle_mod.direct_solve(n, a.reshape(-1), f.reshape(-1)).reshape(n, n)
        errs.append(np.max(np.abs(u - u_ex)))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 3.7), ratios
    assert errs[-1] < 2e-4


def test_layered_medium_second_order(oracle_mod):
    """Coefficient jumping 1 -> 100 across the face x = 1/2, exact solution
    u = sin(2 pi x) sin(pi y) / a(x) (flux a du/dx continuous), f smooth.
    The harmonic face mean keeps O(h^2); an arithmetic mean would drop to
    O(h) (ratio 2), so this pins the face rule."""
    errs = []
    for n in (16, 32, 64, 128):
        c = (np.arange(n) + 0.5) / n
        X, Y = np.meshgrid(c, c, indexing="xy")
        a = np.where(X < 0.5, 1.0, 100.0)
        u_ex = np.sin(2 * np.pi * X) / a * np.sin(np.pi * Y)
        f = 5 * np.pi**2 * np.sin(2 * np.pi * X) * np.sin(np.pi * Y)
        u = oracle_mod.direct_solve(n, a.reshape(-1), f.reshape(-1)).reshape(n, n)
        errs.append(np.max(np.abs(u - u_ex)))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 3.8), ratios


def test_apply_inverts_direct_solve(oracle_mod):
    rng = np.random.default_rng(4)
    for n in (4, 16, 64):
        a = np.exp(rng.standard_normal(n * n))
        f = rng.standard_normal(n * n)
        u = oracle_mod.direct_solve(n, a, f)
        r = f - oracle_mod.apply(n, a, u)
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(f)


def test_operator_symmetric_positive(oracle_mod):
    n = 6
    rng = np.random.default_rng(5)
    a = np.exp(rng.standard_normal(n * n))
    A = np.array([oracle_mod.apply(n, a, e) for e in np.eye(n * n)]).T
    assert np.max(np.abs(A - A.T)) <= 1e-12 * np.max(np.abs(A))
    assert np.min(np.linalg.eigvalsh(0.5 * (A + A.T))) > 0


def test_qoi_definitions(oracle_mod):
    n = 8
    u = np.arange(n * n, dtype=float)
    qm, qc = oracle_mod.qoi(n, u)
    assert qm == u.mean()
    c = n // 2
    cells = [(c - 1) + n * (c - 1), c + n * (c - 1), (c - 1) + n * c, c + n * c]
    assert qc == 0.25 * sum(u[p] for p in cells)


def test_fmg_trace_matches_figure(oracle_mod):
    """FMG figure: mu0 = 1, finest level 3, levels visited
    3,2,1,0,1,0,1,2,1,0,1,2,3,2,1,0,1,2,3 with the recorded (circled)
    solutions at visits 4, 7, 12 and 19."""
    golden = open(__file__.replace("test_oracle_solver.py", "golden/fmg_trace_mu0_1_level3.txt")).read().split()
    want = [int(t) for t in golden[0].split(",")]
    circled = [int(t) for t in golden[1].split(",")]
    P = oracle_mod.Problem(2, 4, 4, 0.3, 1.0, mu0=1)
    r = P.fmg(3, np.ones(P.field_size(3)), trace_cap=100)
    assert r["trace"] == want
    assert [i + 1 for i, m in enumerate(r["marks"]) if m] == circled


def _lognormal_fields(oracle_mod, P, k, count, seed):
    rng = np.random.default_rng(seed)
    return [P.field(rng.standard_normal(P.s), k) for _ in range(count)]


@pytest.mark.parametrize("cfg", ["mlmc_fp64_s10", "mlqmc_fp64_s100"])
def test_fmg_rtol_matches_direct(oracle_mod, cfg):
    w = synth.workload(cfg)
    P = oracle_mod.Problem(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"],
                           mu0=w["mu0"], mu1=w["mu1"], mu2=w["mu2"], rtol=1e-12, max_iters=40)
    k = 2 if w["n0"] == 16 else 4
    for z in _lognormal_fields(oracle_mod, P, k, 3, 17):
        fm = P.sample_from_field(k, z, 0)
        dr = P.sample_from_field(k, z, 1)
        assert fm["status"] == 0
        assert np.all(fm["relres"] <= 1e-12)
        rel = np.abs(fm["qoi"] - dr["qoi"]) / np.abs(dr["qoi"])
        assert np.max(rel) <= 1e-10, rel


def test_fmg_rtol_high_contrast(oracle_mod):
    """sigma^2 = 2, lambda = 0.1: FMG refinement still meets 1e-10 against the
    direct solve, in few flexible-CG steps."""
    P = oracle_mod.Problem(4, 6, 400, 0.1, 2.0, mu0=1, mu1=2, mu2=2, rtol=1e-10, max_iters=40)
    k = 4
    for z in _lognormal_fields(oracle_mod, P, k, 2, 23):
        fm = P.sample_from_field(k, z, 0)
        dr = P.sample_from_field(k, z, 1)
        assert fm["status"] == 0
        assert np.max(fm["iters"]) <= 25
        rel = np.abs(fm["qoi"] - dr["qoi"]) / np.abs(dr["qoi"])
        assert np.max(rel) <= 1e-9, rel


def test_fmg_rtol_rough_lattice_samples_all_converge(oracle_mod):
    """The s = 400, lambda = 0.1, sigma^2 = 2 lattice workload: coarse grids
    (h >= lambda) see coefficients that the rediscretised coarse operators
    represent badly, and plain V-cycle iteration on the residual diverges for
    a sizeable share of these samples (roughly one in five at 16^2 and 32^2).
    V-cycle-preconditioned flexible CG converges on every sample, and each
    converged stage agrees with the band Cholesky solve."""
    w = synth.workload("mlqmc_mixed_s400")
    P = oracle_mod.Problem(w["n0"], 4, w["s"], w["corr_len"], w["sigma2"], mu0=w["mu0"],
                           mu1=w["mu1"], mu2=w["mu2"], rtol=w["rtol"], max_iters=w["max_iters"])
    zv = synth.korobov_vector(w["seed"], w["s"])
    D = synth.shift_table(w["seed"], w["num_levels"], w["num_shifts"], w["s"])
    for k in range(4):
        _, y = oracle_mod.points(zv, D[k, 0], 0, 96)
        worst_it = 0
        for b in range(len(y)):
            z = P.field(y[b], k)
            fm = P.sample_from_field(k, z, 0)
            assert fm["status"] == 0, (k, b, fm)
            assert np.all(fm["relres"][1:] <= w["rtol"])
            worst_it = max(worst_it, int(np.max(fm["iters"])))
            if b % 8 == 0:
                dr = P.sample_from_field(k, z, 1)
                rel = np.abs(fm["qoi"] - dr["qoi"]) / np.abs(dr["qoi"])
                assert np.max(rel) <= 1e-8, (k, b, rel)
        assert worst_it <= 30, (k, worst_it)


def test_fmg_fixed_cycles_reach_discretisation_accuracy(oracle_mod):
    """Two V(2,2) cycles per FMG stage leave an algebraic error below the
    discretisation error: for the mean of u, a quarter of the level
    difference of the direct solves; for both QoIs, an algebraic error that
    shrinks with h like the discretisation error (>= 2x per level)."""
    w = synth.workload("mlqmc_fp64_s100")
    P = oracle_mod.Problem(w["n0"], w["num_levels"], w["s"], w["corr_len"], w["sigma2"])
    k = 5
    for z in _lognormal_fields(oracle_mod, P, k, 3, 29):
        fm = P.sample_from_field(k, z, 0)["qoi"]
        dr = P.sample_from_field(k, z, 1)["qoi"]
        for l in range(1, k + 1):
            assert abs(fm[l, 0] - dr[l, 0]) <= 0.25 * abs(dr[l, 0] - dr[l - 1, 0]), (l, fm[l], dr[l])
        alg = np.abs(fm - dr)
        assert np.all(alg[k] <= alg[1] / 2 ** (k - 1)), alg


def test_fmg_constant_coefficient_matches_series_order(oracle_mod):
    """a = 1 through FMG: QoI within discretisation error of the series."""
    mean, ctr = series_values()
    P = oracle_mod.Problem(4, 6, 4, 0.3, 0.0)
    k = 5
    r = P.sample_from_field(k, np.zeros(P.field_size(k)), 0)
    n = 4 << k
    assert abs(r["qoi"][k, 0] - mean) < 3.0 * 0.53 / n**2
    assert abs(r["qoi"][k, 1] - ctr) < 3.0 * 0.23 / n**2


def test_vcycle_convergence_is_mesh_independent(oracle_mod):
    """a = 1: refinement to 1e-12 takes the same few V(2,2)-preconditioned
    steps on every level (h-independent multigrid convergence)."""
    P = oracle_mod.Problem(4, 7, 4, 0.3, 0.0, mu0=1, mu1=2, mu2=2, rtol=1e-12, max_iters=60)
    r = P.sample_from_field(6, np.zeros(P.field_size(6)), 0)
    assert r["status"] == 0
    its = r["iters"][1:]
    assert np.all(its <= 13) and its.max() - its.min() <= 2, its


def test_fmg_rtol_stops_at_rounding_floor(oracle_mod):
    """An unattainable rtol: every stage stops once four CG steps in a row
    fail to bring the residual ratio 10% below its best value, well before
    max_iters, flagged as not converged; the iterate is then as accurate as
    FP64 allows (the band Cholesky solve agrees to 1e-12)."""
    P = oracle_mod.Problem(4, 5, 100, 0.3, 1.0, mu0=1, mu1=2, mu2=2, rtol=1e-30, max_iters=200)
    k = 4
    for z in _lognormal_fields(oracle_mod, P, k, 2, 31):
        fm = P.sample_from_field(k, z, 0)
        dr = P.sample_from_field(k, z, 1)
        assert fm["status"] != 0
        assert np.all(fm["iters"][1:] >= 4) and np.all(fm["iters"] < 60), fm["iters"]
        assert np.all(fm["relres"][1:] <= 1e-13), fm["relres"]
        rel = np.abs(fm["qoi"] - dr["qoi"]) / np.abs(dr["qoi"])
        assert np.max(rel) <= 1e-12, rel
