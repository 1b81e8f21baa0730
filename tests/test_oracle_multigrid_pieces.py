"""Direct pins of the oracle's V-cycle pieces (Section 4, two-grid correction
scheme and V-cycle; readings: red-black Gauss-Seidel with red first before the
coarse-grid correction and black first after it, restriction by the mean of
the four children, bilinear prolongation with odd reflection at the walls).

Each piece is compared with a dense matrix built here from its definition:
the restriction and the prolongation as Kronecker products of 1-D operators,
each half-sweep of the smoother as a forward triangular solve on the colour
permutation of the matrix that the (separately pinned) operator assembles from
unit vectors, and the V-cycle as the recursion of these dense pieces.  Every
pin also checks that it tells the reading apart from the plausible mistakes
(even reflection, swapped 3/4 and 1/4 weights, sum instead of mean, the other
colour first): each planted mistake, applied to the dense model, must move the
result by far more than the tolerance."""
import numpy as np
import pytest
from scipy.linalg import solve_triangular


def restrict_1d(nc, scale=0.5):
    R = np.zeros((nc, 2 * nc))
    for I in range(nc):
        R[I, 2 * I] = R[I, 2 * I + 1] = scale
    return R


def prolong_1d(nc, reflect=-1.0, near=0.75):
    """Fine cell 2I+a (a = 0, 1) takes `near` of coarse cell I and 1 - near of
    its neighbour on the same side (I-1 for a = 0, I+1 for a = 1); a
    neighbour beyond the wall is coarse cell I reflected with sign
    `reflect`."""
    n = 2 * nc
    P = np.zeros((n, nc))
    for i in range(n):
        I, side = i // 2, (1 if i % 2 else -1)
        P[i, I] += near
        if 0 <= I + side < nc:
            P[i, I + side] += 1.0 - near
        else:
            P[i, I] += reflect * (1.0 - near)
    return P


def dense_R(nc, scale=0.5):
    R1 = restrict_1d(nc, scale)
    return np.kron(R1, R1)


def dense_P(nc, reflect=-1.0, near=0.75):
    # flat index i + n j: kron(P_y, P_x) with both factors the same 1-D matrix
    P1 = prolong_1d(nc, reflect, near)
    return np.kron(P1, P1)


def dense_A(oracle_mod, n, a):
    return np.array([oracle_mod.apply(n, a, e) for e in np.eye(n * n)]).T


def colour_perm(n, first):
    p = np.arange(n * n)
    c = ((p % n) + (p // n)) % 2
    return np.concatenate([p[c == first], p[c != first]])


def gs_sweep(A, f, u, first):
    """One forward Gauss-Seidel sweep with the cells of colour `first` (0 red,
    1 black) ordered before the others: lower-triangular solve on the
    permuted matrix."""
    n = int(round(np.sqrt(A.shape[0])))
    perm = colour_perm(n, first)
    Ap = A[np.ix_(perm, perm)]
    L = np.tril(Ap)
    up = solve_triangular(L, f[perm] - (Ap - L) @ u[perm], lower=True)
    out = np.empty_like(u)
    out[perm] = up
    return out


def dense_vcycle(As, g, u, f, mu1, mu2, pre_first=0, post_first=1, reflect=-1.0, near=0.75,
                 rscale=0.5):
    if g == 0:
        return np.linalg.solve(As[0], f)
    n = 2 << g
    nc = n // 2
    for _ in range(mu1):
        u = gs_sweep(As[g], f, u, pre_first)
    r = f - As[g] @ u
    fc = dense_R(nc, rscale) @ r
    ec = dense_vcycle(As, g - 1, np.zeros(nc * nc), fc, mu1, mu2, pre_first, post_first,
                      reflect, near, rscale)
    u = u + dense_P(nc, reflect, near) @ ec
    for _ in range(mu2):
        u = gs_sweep(As[g], f, u, post_first)
    return u


def coarse_centres(nc):
    c = (np.arange(nc) + 0.5) / nc
    X, Y = np.meshgrid(c, c, indexing="xy")        # X varies along i (fastest)
    return X.reshape(-1), Y.reshape(-1)


@pytest.mark.parametrize("nc", [1, 2, 4, 8])
def test_restriction_is_mean_of_four_children(oracle_mod, nc):
    rng = np.random.default_rng(nc)
    n = 2 * nc
    r = rng.standard_normal(n * n)
    fc = oracle_mod.restrict(nc, r)
    blocks = r.reshape(nc, 2, nc, 2).mean(axis=(1, 3)).reshape(-1)
    assert np.max(np.abs(fc - blocks)) <= 1e-15 * np.max(np.abs(r))
    assert np.max(np.abs(fc - dense_R(nc) @ r)) <= 1e-15 * np.max(np.abs(r))
    # the sum of the children (a plausible slip) is four times larger
    assert np.max(np.abs(fc - dense_R(nc, 1.0) @ r)) > 0.5 * np.max(np.abs(fc))


@pytest.mark.parametrize("nc", [2, 4, 8])
def test_prolongation_reproduces_affine_functions_inside(oracle_mod, nc):
    """Bilinear interpolation with weights (9,3,3,1)/16 is exact for affine
    functions on every fine cell whose four coarse neighbours are inside."""
    n = 2 * nc
    Xc, Yc = coarse_centres(nc)
    Xf, Yf = coarse_centres(n)
    e = 0.3 - 1.7 * Xc + 2.9 * Yc
    want = 0.3 - 1.7 * Xf + 2.9 * Yf
    got = oracle_mod.prolong(nc, e)
    i, j = np.arange(n * n) % n, np.arange(n * n) // n
    inner = (i >= 1) & (i <= n - 2) & (j >= 1) & (j <= n - 2)
    assert np.max(np.abs(got - want)[inner]) <= 1e-14
    # swapped weights (1/4 on the near coarse cell) do not reproduce it
    wrong = dense_P(nc, near=0.25) @ e
    assert np.max(np.abs(wrong - want)[inner]) > 0.1


@pytest.mark.parametrize("nc", [2, 4, 8])
def test_prolongation_walls_are_odd_reflections(oracle_mod, nc):
    """x*y is odd across the walls x = 0 and y = 0, (1-x)(1-y) across x = 1
    and y = 1: with odd reflection the bilinear interpolant reproduces each
    exactly up to those walls (a product of affine functions); an even
    reflection does not."""
    n = 2 * nc
    Xc, Yc = coarse_centres(nc)
    Xf, Yf = coarse_centres(n)
    i, j = np.arange(n * n) % n, np.arange(n * n) // n
    for ec, ef, keep in ((Xc * Yc, Xf * Yf, (i <= n - 2) & (j <= n - 2)),
                         ((1 - Xc) * (1 - Yc), (1 - Xf) * (1 - Yf), (i >= 1) & (j >= 1))):
        got = oracle_mod.prolong(nc, ec)
        assert np.max(np.abs(got - ef)[keep]) <= 1e-14
        even = dense_P(nc, reflect=1.0) @ ec
        assert np.max(np.abs(even - ef)[keep]) > 0.1 / n


@pytest.mark.parametrize("nc", [1, 2, 4, 8])
def test_prolongation_equals_dense_operator(oracle_mod, nc):
    rng = np.random.default_rng(100 + nc)
    e = rng.standard_normal(nc * nc)
    u = rng.standard_normal(4 * nc * nc)
    Pd = dense_P(nc)
    assert np.max(np.abs(oracle_mod.prolong(nc, e) - Pd @ e)) <= 1e-14
    assert np.max(np.abs(oracle_mod.prolong(nc, e, out=u) - (u + Pd @ e))) <= 1e-14


def _lognormal(rng, n, sigma=1.0):
    return np.exp(sigma * rng.standard_normal(n * n))


@pytest.mark.parametrize("n", [4, 8, 16])
def test_half_sweeps_are_gauss_seidel_on_the_colour_permutation(oracle_mod, n):
    """Red then black half-sweeps = one forward Gauss-Seidel sweep over the
    matrix with red cells ordered first; the other order differs."""
    rng = np.random.default_rng(7 * n)
    a = _lognormal(rng, n)
    f = rng.standard_normal(n * n)
    u0 = rng.standard_normal(n * n)
    A = dense_A(oracle_mod, n, a)
    rb = oracle_mod.rb_sweep(n, a, f, oracle_mod.rb_sweep(n, a, f, u0, 0), 1)
    want = gs_sweep(A, f, u0, 0)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(rb - want)) <= 1e-12 * scale
    br = oracle_mod.rb_sweep(n, a, f, oracle_mod.rb_sweep(n, a, f, u0, 1), 0)
    assert np.max(np.abs(br - gs_sweep(A, f, u0, 1))) <= 1e-12 * scale
    assert np.max(np.abs(br - want)) > 1e-3 * scale


def _hierarchy(oracle_mod, rng, g, sigma=1.0):
    a = [_lognormal(rng, 2 << l, sigma) for l in range(g + 1)]
    As = [dense_A(oracle_mod, 2 << l, a[l]) for l in range(g + 1)]
    return np.concatenate(a), As


@pytest.mark.parametrize("g", [1, 2, 3])
@pytest.mark.parametrize("mu", [(2, 2), (1, 0), (0, 1), (2, 1), (1, 2)])
def test_vcycle_equals_dense_recursion(oracle_mod, g, mu):
    """One V(mu1, mu2) of the oracle = the dense recursion: mu1 red-first
    sweeps, residual, mean restriction, V-cycle on the coarse grid from zero,
    bilinear odd-reflection correction, mu2 black-first sweeps; exact solve
    on 2x2."""
    rng = np.random.default_rng(31 * g + 3 * mu[0] + mu[1])
    mu1, mu2 = mu
    P = oracle_mod.Problem(2, 4, 4, 0.3, 1.0, mu0=1, mu1=mu1, mu2=mu2)
    a_all, As = _hierarchy(oracle_mod, rng, g)
    n = 2 << g
    f = rng.standard_normal(n * n)
    u0 = rng.standard_normal(n * n)
    got = P.vcycle(g, a_all, u0, f)
    want = dense_vcycle(As, g, u0, f, mu1, mu2)
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


@pytest.mark.parametrize("g", [2, 3])
def test_vcycle_pin_rejects_planted_mistakes(oracle_mod, g):
    """Each plausible misreading, planted in the dense model, moves a V(2,2)
    far outside the tolerance of the pin above."""
    rng = np.random.default_rng(500 + g)
    P = oracle_mod.Problem(2, 4, 4, 0.3, 1.0, mu0=1, mu1=2, mu2=2)
    a_all, As = _hierarchy(oracle_mod, rng, g)
    n = 2 << g
    f = rng.standard_normal(n * n)
    u0 = rng.standard_normal(n * n)
    got = P.vcycle(g, a_all, u0, f)
    scale = np.max(np.abs(got))
    mutants = dict(even_reflection=dict(reflect=1.0), swapped_weights=dict(near=0.25),
                   black_first_pre=dict(pre_first=1), red_first_post=dict(post_first=0),
                   sum_restriction=dict(rscale=1.0))
    for name, kw in mutants.items():
        wrong = dense_vcycle(As, g, u0, f, 2, 2, **kw)
        assert np.max(np.abs(wrong - got)) > 1e-6 * scale, name


def _error_operator(oracle_mod, P, g, a_all):
    n = 2 << g
    zero = np.zeros(n * n)
    return np.array([P.vcycle(g, a_all, e, zero) for e in np.eye(n * n)]).T


# Asymptotic error reduction of one V(2,2) cycle for a = 1 (spectral radius
# of the error propagation operator) on 8^2 .. 128^2: it grows slowly with
# the number of levels (0.113, 0.132, 0.147, 0.154, 0.160 measured), as the
# V-cycle of a cell-centred scheme with mean restriction does, and stays
# well below the two-grid bound 1/4 of the smoother alone.
VCYCLE_FACTOR_BAND = (0.10, 0.17)


def test_vcycle_factor_constant_coefficient(oracle_mod):
    """a = 1: the spectral radius of the oracle's V(2,2) error propagation
    (assembled from unit vectors, f = 0) equals that of the dense recursion,
    differs from that of every planted mistake, and lies in the stated band
    on every grid up to 128^2 (power iteration on the largest ones)."""
    P = oracle_mod.Problem(2, 7, 4, 0.3, 1.0, mu0=1, mu1=2, mu2=2)
    lo, hi = VCYCLE_FACTOR_BAND
    rhos = []
    for g in (2, 3, 4):
        a_all = np.ones(sum((2 << l) ** 2 for l in range(g + 1)))
        E = _error_operator(oracle_mod, P, g, a_all)
        rho = np.max(np.abs(np.linalg.eigvals(E)))
        rhos.append(rho)
        assert lo <= rho <= hi, (g, rho)
        if g <= 3:
            n = 2 << g
            As = [dense_A(oracle_mod, 2 << l, np.ones((2 << l) ** 2)) for l in range(g + 1)]

            def radius(**kw):
                Ed = np.array([dense_vcycle(As, g, e, np.zeros(n * n), 2, 2, **kw)
                               for e in np.eye(n * n)]).T
                return np.max(np.abs(np.linalg.eigvals(Ed)))

            assert abs(radius() - rho) <= 1e-10
            for kw in (dict(reflect=1.0), dict(near=0.25), dict(pre_first=1), dict(post_first=0),
                       dict(rscale=1.0)):
                assert abs(radius(**kw) - rho) > 5e-3, kw
    for g in (5, 6):
        n = 2 << g
        a_all = np.ones(sum((2 << l) ** 2 for l in range(g + 1)))
        e = np.random.default_rng(9).standard_normal(n * n)
        for _ in range(40):
            e2 = P.vcycle(g, a_all, e, np.zeros(n * n))
            fac = np.linalg.norm(e2) / np.linalg.norm(e)
            e = e2 / np.linalg.norm(e2)
        rhos.append(fac)
        assert lo <= fac <= hi, (g, fac)
    assert np.all(np.diff(rhos) >= -1e-3) and np.all(np.diff(rhos) <= 0.025), rhos
