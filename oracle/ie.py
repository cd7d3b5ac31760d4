"""Discretization of the first-kind Laplace volume integral equation.

Section 2.1 of the paper: the integral equation (e:ie) with kernel (e:k),
Nystrom/collocation on a uniform grid with matrix entries (e:a_2d)/(e:a_3d).
The variable-coefficient form follows the model equation (e:int) with a = 0
and b = c (SPD case): A_bc = diag(b) A diag(c).

Conventions (readings where the paper leaves a choice):
* point index g = j1 + n*j2 (+ n^2*j3), x fastest, 0-based j;
* "cell" grid: x_t = (j_t + 1/2) h, h = 1/n (the text's convention, Section 2.1);
* "node" grid (2D only, used to reproduce the printed 2D eigenvalue tables):
  x_t = j_t/(n-1), off-diagonal weight h^2 with h = 1/n, diagonal = cell integral at h = 1/n;
* the singular self-cell integral is evaluated in closed form (self_cell_integral).
"""
import numpy as np

GRID_CELL = 0
GRID_NODE = 1


def kernel(d, r):
    """Laplace fundamental solution K(r) of (e:k): -(1/2pi) log r in 2D, 1/(4 pi r) in 3D."""
    r = np.asarray(r, dtype=np.float64)
    if d == 2:
        return -np.log(r) / (2.0 * np.pi)
    if d == 3:
        return 1.0 / (4.0 * np.pi * r)
    raise ValueError("d must be 2 or 3")


def self_cell_integral(d, h):
    """Exact integral of K over the cell [-h/2, h/2]^d (diagonal of (e:a_2d)/(e:a_3d)).

    The paper asks for "a proper singular quadrature" without naming one; the
    integral has a closed form.  2D, with a = h/2, the integral of log sqrt(x^2+y^2)
    over [0,a]^2 is a^2 (ln a + ln(2)/2 - 3/2 + pi/4); times 4 and -1/(2 pi) gives
        -(h^2 / 2 pi) (ln h - ln(2)/2 - 3/2 + pi/4).
    3D: the integral of 1/(4 pi r) over the cube [-h/2,h/2]^3 equals
        (3 h^2 / 4 pi) (ln(2 + sqrt 3) - pi/6).
    Pinned against adaptive quadrature in the tests.
    """
    if d == 2:
        return -(h * h / (2.0 * np.pi)) * (np.log(h) - 0.5 * np.log(2.0) - 1.5 + np.pi / 4.0)
    if d == 3:
        return (3.0 * h * h / (4.0 * np.pi)) * (np.log(2.0 + np.sqrt(3.0)) - np.pi / 6.0)
    raise ValueError("d must be 2 or 3")


def grid_points(d, n, grid=GRID_CELL):
    """Collocation points, shape (N, d), index g = j1 + n j2 (+ n^2 j3) (Section 2.1)."""
    if grid == GRID_CELL:
        x1 = (np.arange(n, dtype=np.float64) + 0.5) / n
    elif grid == GRID_NODE:
        if d != 2:
            raise ValueError("node grid is a 2D-table convention only")
        x1 = np.arange(n, dtype=np.float64) / (n - 1)
    else:
        raise ValueError("unknown grid")
    axes = np.meshgrid(*([x1] * d), indexing="ij")
    # meshgrid 'ij' gives axes[t][j1, j2, ...]; flatten with j1 fastest
    return np.stack([a.transpose().reshape(-1) for a in axes], axis=1)


class Problem:
    """Discretized operator A_bc = diag(b) A diag(c) on an n^d grid (Section 2.1, (e:int)).

    b, c: coefficient arrays of length N, or None for 1.
    """

    def __init__(self, d, n, grid=GRID_CELL, b=None, c=None):
        self.d, self.n, self.grid = d, n, grid
        self.N = n ** d
        self.h = 1.0 / n
        self.x = grid_points(d, n, grid)
        self.b = np.ones(self.N) if b is None else np.asarray(b, dtype=np.float64)
        self.c = np.ones(self.N) if c is None else np.asarray(c, dtype=np.float64)
        self.weight = self.h ** d
        self.a_self = self_cell_integral(d, self.h)

    def diag(self):
        """Diagonal entries b_i c_i A_ii."""
        return self.b * self.c * self.a_self

    def block(self, rows, cols):
        """Dense submatrix A_bc[rows, cols], entries of (e:a_2d)/(e:a_3d) with coefficients."""
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        diff = self.x[rows][:, None, :] - self.x[cols][None, :, :]
        r = np.sqrt(np.sum(diff * diff, axis=2))
        same = rows[:, None] == cols[None, :]
        r = np.where(same, 1.0, r)
        a = self.weight * kernel(self.d, r)
        a = np.where(same, self.a_self, a)
        return self.b[rows][:, None] * a * self.c[cols][None, :]

    def dense(self):
        """The full N x N matrix (small N only)."""
        idx = np.arange(self.N)
        return self.block(idx, idx)
