"""Seeded input vectors for the matrix-vector product (no method arithmetic)."""

import numpy as np


def uniform_vector(n: int, seed: int = 1) -> np.ndarray:
    """x ~ U[-1, 1] in FP64, from numpy's default_rng(seed)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def gaussian_block(n: int, nrhs: int, seed: int = 2) -> np.ndarray:
    """X ~ N(0, 1), n x nrhs, column-major (Fortran order), FP64."""
    g = np.random.default_rng(seed).standard_normal((nrhs, n))
    return np.asfortranarray(g.T)
