"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method itself: it only draws the
right-hand sides and evaluates the smooth coefficient field at grid points.
Both the oracle and the HIP path receive the arrays it returns.
"""
import numpy as np


def rhs(N, nrhs=1, seed=0):
    """Right-hand sides f ~ N(0,1): array of shape (nrhs, N), row j = RHS j.

    Drawn with numpy's default_rng(seed).standard_normal((nrhs, N)), so the
    first row is the same whatever nrhs is.
    """
    return np.random.default_rng(seed).standard_normal((nrhs, N))


def cell_centres_1d(n):
    """Cell-centre coordinates (j + 1/2)/n, j = 0..n-1, of the unit interval."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def coef_smooth(d, n):
    """Smooth positive coefficient b = c = 1 + 0.5 sin(2 pi x1) cos(2 pi x2).

    Evaluated at the cell centres of the n^d grid, point index
    j1 + n*j2 (+ n^2*j3) (x fastest).  In 3D the field does not depend on x3.
    Values lie in [0.5, 1.5].
    """
    x = cell_centres_1d(n)
    f2 = 1.0 + 0.5 * np.outer(np.cos(2 * np.pi * x), np.sin(2 * np.pi * x))
    # f2[j2, j1] = 1 + 0.5 sin(2 pi x_{j1}) cos(2 pi x_{j2})
    if d == 2:
        return np.ascontiguousarray(f2.reshape(-1))
    return np.ascontiguousarray(np.broadcast_to(f2, (n, n, n)).reshape(-1))
