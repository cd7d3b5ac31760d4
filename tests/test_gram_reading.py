"""The reading behind CBD_ID_GRAM: the truncated pivoted Cholesky of G = Y^T Y makes
the choices of the truncated column-pivoted QR of Y ((e:id), Section 4.2).

After j steps the Schur-complement diagonal of G is the squared norm of each column
of Y with its projection on the chosen columns removed, which is the trailing-block
column norm the QR compares; the Cholesky factor is R^T up to row signs, and
T = R11^{-1} R12 does not see the signs.  In FP64 the squared norms carry a rounding
floor near 1e-16 |Y|^2, so the equality is checked at tolerances >= 1e-7.  The
pivoted Cholesky here is written for the test (no GPU, no library code)."""
import numpy as np
import pytest
from scipy.linalg import solve_triangular

from oracle import dd, ie, rs
from oracle.cpqr import TIE_FP64, interp_decomp


def pivoted_cholesky_id(Y, tol, tie=TIE_FP64):
    G = Y.T @ Y
    n = G.shape[1]
    kmax = min(Y.shape)
    d = np.diag(G).copy()
    pv = np.arange(n)
    L = np.zeros((n, kmax))
    rdiag = np.zeros(kmax)
    nu0, k = None, kmax
    for j in range(kmax):
        norms = np.sqrt(np.maximum(d[pv[j:]], 0.0))
        mx = norms.max()
        if nu0 is None:
            nu0 = mx
        if nu0 == 0.0 or mx <= tol * nu0:
            k = j
            break
        P = j + int(np.argmax(norms >= mx - tie * nu0))   # lowest position in the window
        p = pv[P]
        rdiag[j] = np.sqrt(d[p])
        rest = pv[j:][pv[j:] != p]
        L[rest, j] = (G[rest, p] - L[rest, :j] @ L[p, :j]) / rdiag[j]
        d[rest] -= L[rest, j] ** 2
        pv[j], pv[P] = p, pv[j]
    R = np.zeros((k, n))
    for j in range(k):
        R[j, j] = rdiag[j]
        R[j, j + 1:] = L[pv[j + 1:], j]
    T = solve_triangular(R[:, :k], R[:, k:], lower=False) if k else np.zeros((0, n))
    return k, pv, T


def _boxes():
    """Proxy matrices of leaf boxes of a 64^2 CBD subdomain (m = 16) and of its
    first-level parents (active DOFs: the leaves' oracle skeletons)."""
    prob = ie.Problem(2, 64)
    part = dd.Partition(2, 64, 16, 1, dd.CBD)
    sd = part.subdomains[1]
    f = rs.factor_subdomain(prob, part, sd, 1e-6)
    out = []
    allp = np.arange(len(sd.index))
    for bi in (0, 5, 22, 63):
        st, cnt = sd.leaves[bi][2], sd.leaves[bi][3]
        p = np.arange(st, st + cnt)
        out.append(rs.proxy_matrix(prob, sd, sd.levels[0][bi], p, np.setdiff1d(allp, p))[0])
    act = [np.concatenate([f.levels[0][c].sk for c in box.children]) for box in sd.levels[1]]
    allact = np.concatenate(act)
    for bi in (0, 7, 15):
        out.append(rs.proxy_matrix(prob, sd, sd.levels[1][bi], act[bi], np.setdiff1d(allact, act[bi]))[0])
    return out


BOXES = _boxes()


@pytest.mark.parametrize("tol", [1e-3, 1e-6])
def test_pivoted_cholesky_of_the_gram_matrix_is_the_qr_id(tol):
    for bi, Y in enumerate(BOXES):
        k, perm, T = interp_decomp(Y, tol)
        kc, pc, Tc = pivoted_cholesky_id(Y, tol)
        assert kc == k and np.array_equal(pc, perm), (bi, k, kc)
        if k and k < Y.shape[1]:
            # T agrees to about u cond(R11)^2 <= u / tol^2 relative
            assert np.linalg.norm(Tc - T) <= max(1e-10, 1e-15 / tol ** 2) * 100 * np.linalg.norm(T), bi
            # and both IDs leave residual columns within the QR's stopping bound
            nu0 = np.linalg.norm(Y, axis=0).max()
            for TT, pp in ((T, perm), (Tc, pc)):
                res = Y[:, pp[k:]] - Y[:, pp[:k]] @ TT
                assert np.linalg.norm(res, axis=0).max() <= 1.01 * tol * nu0, bi
