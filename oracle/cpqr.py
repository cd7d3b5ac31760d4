"""Interpolative decomposition by truncated column-pivoted QR.

Section 4.2, (e:id)/(e:id_err): the columns p of a block are split into
skeletons s and redundant columns r with A_{qr} ~= A_{qs} T.  The paper cites
Cheng et al. for the ID; that construction is a column-pivoted (Businger-Golub)
QR: at each step the column with the largest remaining 2-norm is moved to the
front and eliminated with a Householder reflection.  With Y[:, perm] = Q R,
T = R11^{-1} R12.

Readings (where the paper leaves a choice):
* rank rule: stop at the first step j whose largest remaining column norm is
  <= tol * (largest column norm of Y); k = j.  All-zero Y gives k = 0;
* column norms are recomputed from the remaining block at every step (no
  down-dating);
* tie rule: among columns whose remaining norm is within tie * (largest column
  norm of Y) of the maximum, the lowest current position wins.  The grids
  here are symmetric, so exact ties are common and both implementations must
  break them the same way;
* the redundant columns keep the order that the column swaps leave them in.
"""
import numpy as np
from scipy.linalg import solve_triangular

TIE_FP64 = 1e-10


def cpqr_truncated(Y, tol, tie=TIE_FP64):
    """Truncated CPQR.  Returns (k, perm, R) with R the k x n upper-trapezoidal factor
    in permuted column order (R = Q^T Y[:, perm] restricted to its first k rows)."""
    A = np.array(Y, dtype=np.float64, copy=True)
    m, n = A.shape
    perm = np.arange(n)
    k = 0
    nu0 = 0.0
    for j in range(min(m, n)):
        norms = np.sqrt(np.sum(A[j:, j:] ** 2, axis=0))
        mx = norms.max()
        if j == 0:
            nu0 = mx
            if nu0 == 0.0:
                break
        if mx <= tol * nu0:
            break
        cand = int(np.nonzero(norms >= mx - tie * nu0)[0][0])
        piv = j + cand
        if piv != j:
            A[:, [j, piv]] = A[:, [piv, j]]
            perm[[j, piv]] = perm[[piv, j]]
        x = A[j:, j].copy()
        xn = np.sqrt(np.sum(x * x))
        alpha = -xn if x[0] >= 0 else xn
        v = x
        v[0] -= alpha
        vn = np.sqrt(np.sum(v * v))
        if vn > 0:
            v /= vn
            A[j:, j:] -= 2.0 * np.outer(v, v @ A[j:, j:])
        A[j, j] = alpha
        A[j + 1:, j] = 0.0
        k = j + 1
    R = np.triu(A[:k, :])
    return k, perm, R


def interp_decomp(Y, tol, tie=TIE_FP64):
    """ID of the columns of Y: returns (k, perm, T) with Y[:, perm[k:]] ~= Y[:, perm[:k]] @ T."""
    k, perm, R = cpqr_truncated(Y, tol, tie)
    n = Y.shape[1]
    if k == 0:
        return 0, perm, np.zeros((0, n))
    T = solve_triangular(R[:, :k], R[:, k:], lower=False)
    return k, perm, T
