"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

Holds no arithmetic of the transform itself: only random numbers laid out in the
coefficient order omega(n,l,m) = n(n-1)(2n-1)/6 + l(l+1) + m and the sample order
psi(i,j,k) = 4B^2 i + 2B j + k (Sect. 3.4 of the paper), whose index maps it
needs to know the degree n of each coefficient.

Distributions
  * complex normal CN(0,1): (x + i y)/sqrt(2), x, y ~ N(0,1), so E|z|^2 = 1;
    optionally times n^-p with n the coefficient's degree (decaying spectrum);
  * the paper's own protocol (Sect. 4): real and imaginary parts ~ U(-1, 1);
  * random (not bandlimited) complex normal samples.
Generator: numpy PCG64 seeded with an integer; one stream per call.
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 160405140


def num_coeffs(B: int) -> int:
    return B * (B + 1) * (2 * B + 1) // 6


def num_samples(B: int) -> int:
    return 8 * B ** 3


def degree_of_each_coeff(B: int) -> np.ndarray:
    """n for every omega index (degree n owns n^2 consecutive slots)."""
    return np.repeat(np.arange(1, B + 1), np.arange(1, B + 1) ** 2)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def complex_normal_coeffs(B: int, batch: int = 1, seed: int = BASE_SEED, decay: float = 0.0) -> np.ndarray:
    """(batch, Omega) complex128, CN(0,1) * n^-decay."""
    g = _rng(seed)
    om = num_coeffs(B)
    z = (g.standard_normal((batch, om)) + 1j * g.standard_normal((batch, om))) / np.sqrt(2.0)
    if decay:
        z = z * degree_of_each_coeff(B)[None, :].astype(np.float64) ** (-decay)
    return z


def uniform_coeffs(B: int, batch: int = 1, seed: int = BASE_SEED) -> np.ndarray:
    """(batch, Omega) complex128 with Re, Im ~ U(-1, 1) (the paper's Sect. 4 protocol)."""
    g = _rng(seed)
    om = num_coeffs(B)
    return g.uniform(-1, 1, (batch, om)) + 1j * g.uniform(-1, 1, (batch, om))


def complex_normal_samples(B: int, batch: int = 1, seed: int = BASE_SEED) -> np.ndarray:
    """(batch, 8B^3) complex128 CN(0,1) samples (not bandlimited)."""
    g = _rng(seed)
    ps = num_samples(B)
    return (g.standard_normal((batch, ps)) + 1j * g.standard_normal((batch, ps))) / np.sqrt(2.0)


def subset(count: int, total: int, seed: int) -> np.ndarray:
    """Sorted distinct indices in [0, total)."""
    g = _rng(seed)
    count = min(count, total)
    return np.sort(g.choice(total, size=count, replace=False))


def grid_points(count: int, B: int, seed: int) -> np.ndarray:
    """(count, 3) distinct (i, j, k) grid triples."""
    flat = subset(count, num_samples(B), seed)
    n2 = 2 * B
    return np.stack([flat // (n2 * n2), (flat // n2) % n2, flat % n2], axis=1)


def batched_bandlimits(nfunc: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """nfunc bandlimits drawn uniformly from {lo, ..., hi}."""
    return _rng(seed).integers(lo, hi + 1, size=nfunc)
