"""Seeded coefficient vectors and materials."""

from __future__ import annotations

import numpy as np


def n_basis(N: int) -> int:
    """Number of basis functions of degree N on the pyramid: sum_k (k+1)^2."""
    return (N + 1) * (N + 2) * (2 * N + 3) // 6


def random_state(K: int, N: int, seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Standard-normal coefficients in the canonical layout (K, 4, Np): p, u, v, w."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((K, 4, n_basis(N)))


def random_materials(K: int, seed: int = 0, lo: float = 0.5, hi: float = 2.0):
    """Piecewise-constant density and bulk modulus, each uniform in [lo, hi]."""
    rng = np.random.default_rng(seed + 104729)
    rho = rng.uniform(lo, hi, K)
    kappa = rng.uniform(lo, hi, K)
    return rho, kappa
