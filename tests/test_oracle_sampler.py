"""Pins of the oracle's sampler (Section 3.2: randomly shifted rank-1 lattice
rule used as a lattice sequence, mapped through the inverse normal CDF)
against facts fixed by the mathematics and by library routines."""
import numpy as np
import pytest
import scipy.special as sp

import synth


def test_bitrev32_brute_force(oracle_mod):
    rng = np.random.default_rng(0)
    for v in list(rng.integers(0, 2**32, 200)) + [0, 1, 2**31, 2**32 - 1, 0x12345678]:
        v = int(v)
        want = int(format(v, "032b")[::-1], 2)
        assert oracle_mod.bitrev32(v) == want


def test_korobov_vector_properties():
    for seed in range(5):
        a = synth.korobov_multiplier(seed)
        assert a % 8 in (3, 5)
        z = synth.korobov_vector(seed, 300)
        assert z[0] == 1 and np.all(z % 2 == 1)
        for m in (10, 12):
            zm = z.astype(np.int64) % (1 << m)
            # maximal order 2^(m-2): no repeated component while j <= 2^(m-2)
            assert len(set(zm[: min(300, 1 << (m - 2))].tolist())) == min(300, 1 << (m - 2))


@pytest.mark.parametrize("m", [4, 7, 10])
def test_sequence_prefix_is_lattice_rule(oracle_mod, m):
    """The first 2^m points of the sequence are, as a set, the paper's
    N = 2^m point rule {n z / N}, n = 0..N-1, in natural order."""
    s = 12
    z = synth.korobov_vector(7, s)
    zero = np.zeros(s, dtype=np.uint64)
    N = 1 << m
    seq = {tuple(oracle_mod.lattice_x(z, zero, n).tolist()) for n in range(N)}
    zN = z.astype(np.int64) % N
    rule = set()
    for n in range(N):
        frac = (n * zN) % N                         # {n z / N} * N
        rule.add(tuple((int(f) << (64 - m)) for f in frac))  # as 64-bit fixed point
    assert seq == rule


def test_projections_are_permutations(oracle_mod):
    """Each 1-D projection of the first 2^q points is a permutation of the
    multiples of 2^-q (z_j odd)."""
    s, q = 8, 9
    z = synth.korobov_vector(3, s)
    zero = np.zeros(s, dtype=np.uint64)
    xs = np.array([oracle_mod.lattice_x(z, zero, n) for n in range(1 << q)])
    for j in range(s):
        ks = sorted(int(v) >> (64 - q) for v in xs[:, j])
        assert ks == list(range(1 << q))
        assert all(int(v) % (1 << (64 - q)) == 0 for v in xs[:, j])


def test_shift_is_modular_addition(oracle_mod):
    s = 16
    z = synth.korobov_vector(1, s)
    D = synth.shift_table(1, 2, 3, s)[1, 2]
    zero = np.zeros(s, dtype=np.uint64)
    for n in [0, 1, 5, 1023, 77777]:
        x0 = oracle_mod.lattice_x(z, zero, n)
        x = oracle_mod.lattice_x(z, D, n)
        for j in range(s):
            assert (int(x0[j]) + int(D[j])) % (1 << 64) == int(x[j])
    # n = 0 is the shift itself; n = 1 is the point 1/2 + Delta
    assert np.array_equal(oracle_mod.lattice_x(z, D, 0), D)
    x1 = oracle_mod.lattice_x(z, D, 1)
    assert all((int(D[j]) + (1 << 63)) % (1 << 64) == int(x1[j]) for j in range(s))


def test_unit_map(oracle_mod):
    assert oracle_mod.unit(0) == 2.0**-53
    assert oracle_mod.unit(2**64 - 1) == 1.0 - 2.0**-53
    rng = np.random.default_rng(5)
    for x in rng.integers(0, 2**63, 500, dtype=np.int64):
        x = int(x) * 2 + 1
        u = oracle_mod.unit(x)
        assert 0.0 < u < 1.0
        # bit complement maps to the mirrored point exactly
        assert oracle_mod.unit((2**64 - 1) ^ x) == 1.0 - u
        # u is the centre of the 2^-52 cell containing x / 2^64
        assert abs(u - x / 2.0**64) <= 2.0**-53


def test_norminv_against_library(oracle_mod):
    """Within 2 ulp of a 200-bit evaluation (mpmath) and 4 ulp of scipy."""
    mp = pytest.importorskip("mpmath")
    mp.mp.prec = 200
    rng = np.random.default_rng(11)
    us = list(rng.random(1500)) + [2.0**-53, 1e-10, 0.25, 0.5 - 2.0**-53,
                                   0.5 + 2.0**-53, 0.75, 1 - 2.0**-53, 0.975]
    for u in us:
        y = oracle_mod.norminv(u)
        exact = float(-mp.sqrt(2) * mp.erfinv(1 - 2 * mp.mpf(u)))
        assert abs(y - exact) <= 2 * np.spacing(abs(exact)), (u, y, exact)
        assert abs(y - sp.ndtri(u)) <= 4 * np.spacing(abs(exact)), (u, y)


def test_norminv_identities(oracle_mod):
    # textbook quantile
    assert abs(oracle_mod.norminv(0.975) - 1.959963984540054) <= 2e-15
    assert oracle_mod.norminv(0.5) == 0.0
    rng = np.random.default_rng(12)
    for x in rng.integers(0, 2**63, 300, dtype=np.int64):
        u = oracle_mod.unit(int(x))
        y = oracle_mod.norminv(u)
        # exact symmetry under the mirrored point
        assert oracle_mod.norminv(oracle_mod.unit((2**64 - 1) ^ int(x))) == -y
        # Phi(Phi^-1(u)) = u up to the granularity of y and a few ulp of u
        back = sp.ndtr(y) if u < 0.5 else 1.0 - sp.ndtr(-y)
        pdf = np.exp(-0.5 * y * y) / np.sqrt(2 * np.pi)
        assert abs(back - u) <= 2 * pdf * np.spacing(abs(y)) + 4 * np.spacing(u)


def test_points_batch_matches_scalar(oracle_mod):
    s = 20
    z = synth.korobov_vector(2, s)
    D = synth.shift_table(2, 1, 1, s)[0, 0]
    x, y = oracle_mod.points(z, D, 100, 140)
    for n in (100, 117, 139):
        xs = oracle_mod.lattice_x(z, D, n)
        assert np.array_equal(x[n - 100], xs)
        assert np.array_equal(y[n - 100], [oracle_mod.norminv(oracle_mod.unit(int(v))) for v in xs])
