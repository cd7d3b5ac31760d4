"""Additive preconditioner with exact subdomain solves ("naive" CBD, Section 5.1).

T^{-1} = sum_i R_i^T A_i^{-1} R_i with A_i = R_i A R_i^T (e:ai), (e:ad), each A_i
factored by dense Cholesky.  With oracle.dd modes this gives the block Jacobi,
Schwarz and CBD preconditioners of table t:dd.
"""
import numpy as np
from scipy.linalg import cho_factor, cho_solve


class ExactPreconditioner:
    def __init__(self, prob, part, A=None):
        self.part = part
        self.fac = []
        for sd in part.subdomains:
            Ai = A[np.ix_(sd.index, sd.index)] if A is not None else prob.block(sd.index, sd.index)
            self.fac.append(cho_factor(Ai, lower=False))

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        z = np.zeros_like(r)
        for sd, fc in zip(self.part.subdomains, self.fac):
            z[sd.index] += cho_solve(fc, r[sd.index])
        return z

    def dense(self, N):
        """The N x N matrix T^{-1} (small N only)."""
        Minv = np.zeros((N, N))
        for sd, fc in zip(self.part.subdomains, self.fac):
            Minv[np.ix_(sd.index, sd.index)] += cho_solve(fc, np.eye(len(sd.index)))
        return Minv


def preconditioned_eigenvalues(A, Minv):
    """Eigenvalues of T^{-1} A (e:ta) via the similar symmetric matrix L^T T^{-1} L, A = L L^T."""
    L = np.linalg.cholesky(A)
    S = L.T @ Minv @ L
    return np.linalg.eigvalsh(0.5 * (S + S.T))
