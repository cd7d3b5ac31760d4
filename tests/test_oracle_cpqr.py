"""Pins of the oracle's interpolative decomposition (Section 4.2, (e:id)/(e:id_err))."""
import numpy as np
import pytest
import scipy.linalg

from oracle.cpqr import cpqr_truncated, interp_decomp


@pytest.mark.parametrize("m,n,seed", [(40, 12, 0), (12, 30, 1), (64, 64, 2)])
def test_pivots_match_lapack_on_generic_matrices(m, n, seed):
    # LAPACK dgeqp3 is the same Businger-Golub pivoting; on matrices without ties
    # the pivot sequence and |diag R| must agree
    Y = np.random.default_rng(seed).standard_normal((m, n))
    k, perm, R = cpqr_truncated(Y, tol=0.0)
    Q2, R2, P2 = scipy.linalg.qr(Y, pivoting=True, mode="economic")
    kk = min(m, n)
    assert k == kk
    assert np.array_equal(perm[:kk], P2[:kk])
    assert np.allclose(np.abs(np.diag(R)[:kk]), np.abs(np.diag(R2)), rtol=1e-12)
    # R reproduces Y[:, perm] with an orthogonal Q
    Q = Y[:, perm][:, :k] @ np.linalg.inv(R[:, :k])
    assert np.allclose(Q.T @ Q, np.eye(k), atol=1e-10)


def test_low_rank_matrix_rank_and_exact_reconstruction():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((50, 7)) @ rng.standard_normal((7, 20))
    k, perm, T = interp_decomp(Y, tol=1e-10)
    assert k == 7
    assert np.allclose(Y[:, perm[k:]], Y[:, perm[:k]] @ T, atol=1e-10 * np.abs(Y).max())


def test_rank_rule_threshold():
    # columns with geometric norms and orthogonal directions: R_jj = 10^-j
    Y = np.diag(10.0 ** -np.arange(8))
    for tol, k_expect in [(0.5, 1), (2e-4, 4), (1e-4, 4), (9.9e-5, 5), (0.0, 8)]:
        k, perm, _ = cpqr_truncated(Y, tol)
        assert k == k_expect, (tol, k)
        assert np.array_equal(perm[:k], np.arange(k))


def test_zero_matrix_and_full_rank_edge_cases():
    k, perm, T = interp_decomp(np.zeros((5, 4)), 1e-6)
    assert k == 0 and T.shape == (0, 4)
    k, perm, T = interp_decomp(np.eye(4), 1e-6)
    assert k == 4 and T.shape == (4, 0)


def test_tie_rule_lowest_index_wins():
    # two identical columns: the lower index is the skeleton, the other is
    # reproduced exactly by it
    rng = np.random.default_rng(5)
    a = rng.standard_normal(10)
    b = rng.standard_normal(10) * 0.1
    Y = np.stack([b, a, a, b], axis=1)
    k, perm, T = interp_decomp(Y, 1e-12)
    assert perm[0] == 1
    assert k == 2
    assert perm[1] == 0


def test_id_error_bound():
    # (e:id_err): ||A_qr - A_qs T|| <= eps ||A_qp|| (up to a modest factor)
    rng = np.random.default_rng(11)
    U = rng.standard_normal((80, 30))
    s = 10.0 ** -np.linspace(0, 12, 30)
    Y = (U * s) @ rng.standard_normal((30, 25))
    for tol in (1e-3, 1e-6, 1e-9):
        k, perm, T = interp_decomp(Y, tol)
        err = np.linalg.norm(Y[:, perm[k:]] - Y[:, perm[:k]] @ T, 2)
        assert err <= 30 * tol * np.linalg.norm(Y, 2)
        assert k < 25
