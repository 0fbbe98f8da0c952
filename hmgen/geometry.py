"""Synthetic point sets standing in for the paper's two model problems.

The paper's Laplace single-layer problem lives on the unit sphere and its
Matern covariance problem on random points (Sec. 5.1).  Here the sphere is a
Fibonacci lattice and the covariance problem uses uniform random points in the
unit cube; both are seeded and exactly reproducible.
"""

import math

import numpy as np
from scipy.spatial import cKDTree


def fibonacci_sphere(n: int) -> np.ndarray:
    """n points on the unit sphere: z_i = 1-(2i+1)/n, phi_i = i*pi*(3-sqrt 5)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    phi = i * (math.pi * (3.0 - math.sqrt(5.0)))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.ascontiguousarray(np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1))


def cube_points(n: int, seed: int = 0) -> np.ndarray:
    """n points uniform in [0,1)^3 from numpy's default_rng(seed)."""
    return np.ascontiguousarray(np.random.default_rng(seed).random((n, 3)))


def mean_nn_distance(pts: np.ndarray) -> float:
    """Mean distance from each point to its nearest other point (exact, k-d tree)."""
    d, _ = cKDTree(pts).query(pts, k=2)
    return float(d[:, 1].mean())
