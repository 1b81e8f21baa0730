"""Seeded synthetic inputs for the MG-MLQMC sampler.

This module produces the random draws the method consumes, and nothing else:

* the rank-1 lattice generating vector (Section 3.2 takes it as an external
  input; here it is a Korobov vector whose multiplier is drawn from the seed),
* the random shifts Delta_l^(r), one per (level, shift, dimension),
* i.i.d. N(0,1) vectors for plain Monte Carlo sampling.

It holds none of the method's arithmetic (no lattice points, no inverse normal
map, no field, no solve, no estimator).  Both the oracle tests and the GPU
library take its outputs as inputs, so the two implementations see identical
draws without sharing any code.

The workloads below are the synthetic stand-ins for the paper's experiments
(the paper's own parameter files, Matern fields and generating vector are not
available); every number here is a design choice documented with the build.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "korobov_multiplier",
    "korobov_vector",
    "shift_table",
    "mc_normals",
    "WORKLOADS",
    "workload",
]

_TAG_KOROBOV = 1
_TAG_SHIFT = 2
_TAG_MC = 3


def korobov_multiplier(seed: int) -> int:
    """Odd multiplier a with a = 3 or 5 (mod 8), drawn from the seed.

    Such an a has the largest possible multiplicative order, 2^(m-2), modulo
    2^m, so the components a^(j-1) mod 2^m stay distinct for j <= 2^(m-2).
    """
    rng = np.random.default_rng([int(seed), _TAG_KOROBOV])
    while True:
        a = 2 * int(rng.integers(0, 2**31)) + 1
        if a % 8 in (3, 5):
            return a


def korobov_vector(seed: int, s: int) -> np.ndarray:
    """Generating vector z_j = a^(j-1) mod 2^32, j = 1..s, as uint32.

    Reduced modulo N = 2^m this is the Korobov vector a^(j-1) mod N of an
    N-point rank-1 lattice rule, for every m <= 32.
    """
    a = korobov_multiplier(seed)
    z = np.empty(s, dtype=np.uint32)
    v = 1
    for j in range(s):
        z[j] = v
        v = (v * a) % (1 << 32)
    return z


def shift_table(seed: int, num_levels: int, num_shifts: int, s: int) -> np.ndarray:
    """Uniform random shifts as 64-bit fixed point, shape [levels][shifts][s].

    Entry D[l, r, j] stands for the real number D / 2^64 in [0, 1): the j-th
    component of the shift Delta_l^(r), i.i.d. over l, r and j.
    """
    rng = np.random.default_rng([int(seed), _TAG_SHIFT])
    raw = rng.bit_generator.random_raw(num_levels * num_shifts * s)
    return np.asarray(raw, dtype=np.uint64).reshape(num_levels, num_shifts, s)


def mc_normals(seed: int, level: int, n: int, s: int, replica: int = 0) -> np.ndarray:
    """n i.i.d. standard normal vectors of length s (float64, [n][s])."""
    rng = np.random.default_rng([int(seed), _TAG_MC, int(level), int(replica)])
    return rng.standard_normal((n, s))


# Synthetic workloads.  Grid: level l has n0 * 2^l cells per side on the unit
# square; the field is lognormal with separable exponential covariance.
WORKLOADS = {
    # plain MLMC, FP64, Monte Carlo normals, 16^2 .. 64^2
    "mlmc_fp64_s10": dict(
        n0=16, num_levels=3, s=10, corr_len=0.3, sigma2=1.0,
        mu0=2, mu1=2, mu2=2, rtol=0.0, max_iters=0, precision="fp64",
        qoi=("mean",), sampling="mc", samples_per_level=(256, 64, 16),
        num_shifts=1, seed=1,
    ),
    # MLQMC FP64, Korobov lattice 2^10 points x 16 shifts, 4^2 .. 256^2
    "mlqmc_fp64_s100": dict(
        n0=4, num_levels=7, s=100, corr_len=0.3, sigma2=1.0,
        mu0=2, mu1=2, mu2=2, rtol=0.0, max_iters=0, precision="fp64",
        qoi=("mean", "center"), sampling="lattice", lattice_log2n=10,
        num_shifts=16, seed=2,
    ),
    # mixed precision, 2^12 points x 16 shifts, 4^2 .. 1024^2, refinement to 1e-10
    "mlqmc_mixed_s400": dict(
        n0=4, num_levels=9, s=400, corr_len=0.1, sigma2=2.0,
        mu0=1, mu1=2, mu2=2, rtol=1e-10, max_iters=60, precision="mixed",
        qoi=("mean", "center"), sampling="lattice", lattice_log2n=12,
        num_shifts=16, seed=3,
    ),
    # uneven levels: 4^2 .. 2048^2 with 2^(16-l) samples on level l (65536 ..
    # 128, 130944 in all), the mixed path refined to 1e-10
    "uneven_mixed_s400": dict(
        n0=4, num_levels=10, s=400, corr_len=0.1, sigma2=2.0,
        mu0=1, mu1=2, mu2=2, rtol=1e-10, max_iters=60, precision="mixed",
        qoi=("mean", "center"), sampling="lattice", lattice_log2n=12,
        num_shifts=16, seed=4, samples_per_level=tuple(1 << (16 - l) for l in range(10)),
    ),
    # serving: requests of an adaptive MLQMC driver, s = 1000, lambda 0.05,
    # 4^2 .. 2048^2, FP64 with 2 V(2,2) cycles per FMG stage
    "serving_fp64_s1000": dict(
        n0=4, num_levels=10, s=1000, corr_len=0.05, sigma2=1.0,
        mu0=2, mu1=2, mu2=2, rtol=0.0, max_iters=0, precision="fp64",
        qoi=("mean", "center"), sampling="lattice", lattice_log2n=16,
        num_shifts=16, seed=5,
    ),
}


def workload(name: str) -> dict:
    """A copy of a named workload's parameters."""
    return dict(WORKLOADS[name])
