"""Product with A by FFT, the matvec the paper uses on the uniform grid (Section 5).

Test infrastructure only (see oracle/__init__.py).

On the cell-centred grid of Section 2.1, x_i - x_j = h (j(i) - j(j)) with integer
grid offsets, so the off-diagonal part of (e:a_2d)/(e:a_3d) is a convolution:

    (A_bc x)_i = b_i [ sum_{j != i} h^d K(h |delta_ij|) c_j x_j ] + b_i c_i A_ii x_i,

with delta_ij = grid(i) - grid(j).  The sum is the aperiodic convolution of
c o x with g[delta] = h^d K(h |delta|) (g[0] = 0) over the n^d grid; it is
evaluated exactly (up to rounding) by embedding both in a periodic grid of
2n points per axis, where g at offset delta in [-(n-1), n-1] sits at delta mod 2n
and the offset n is zero, and multiplying their discrete Fourier transforms.
numpy's FFT is the library step.  Pinned in the tests against the dense oracle
matvec (oracle/c/matvec.c), 2D and 3D, with coefficients.
"""
import numpy as np

from . import ie


def _embedded_kernel(prob):
    d, n = prob.d, prob.n
    if prob.grid != ie.GRID_CELL:
        raise ValueError("the FFT product is written for the cell-centred grid")
    P = 2 * n
    off = np.arange(P)
    off = np.where(off < n, off, off - P).astype(np.float64)   # periodic offset in [-n, n)
    off[n] = np.nan            # offset n: never reached from inside the grid; zero for definiteness
    axes = np.meshgrid(*([off] * d), indexing="ij")
    r2 = sum(a * a for a in axes)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = prob.weight * ie.kernel(d, prob.h * np.sqrt(r2))
    g[np.isnan(g)] = 0.0          # the offset-n planes
    g[(0,) * d] = 0.0             # delta = 0: the diagonal is added separately
    return g


class FFTMatvec:
    """y = A_bc x for x of shape (N,) or (N, nrhs), via one circulant embedding."""

    def __init__(self, prob):
        self.prob = prob
        self.ghat = np.fft.rfftn(_embedded_kernel(prob))

    def __call__(self, X):
        prob = self.prob
        d, n = prob.d, prob.n
        X = np.asarray(X, dtype=np.float64)
        one = X.ndim == 1
        Xc = X[:, None] if one else X
        P = 2 * n
        Y = np.empty_like(Xc)
        shape = (n,) * d                       # C order: last axis is x1 (the fastest index)
        for c in range(Xc.shape[1]):
            v = (prob.c * Xc[:, c]).reshape(shape)
            pad = np.zeros((P,) * d)
            pad[(slice(0, n),) * d] = v
            conv = np.fft.irfftn(np.fft.rfftn(pad) * self.ghat, s=(P,) * d)
            y = conv[(slice(0, n),) * d].reshape(-1)
            Y[:, c] = prob.b * y + prob.b * prob.c * prob.a_self * Xc[:, c]
        return Y[:, 0] if one else Y
