"""Pins of the oracle's PCG (Section 5) against textbook properties of
conjugate gradients that do not depend on its own recurrences.

* The j-th CG iterate from x0 = 0 minimises the A-norm of the error over the
  Krylov space K_j(A, f), so it equals the Galerkin projection onto that space,
  computed here from an explicit orthonormal basis.
* In exact arithmetic CG ends after as many steps as A has distinct
  eigenvalues. With an SPD preconditioner M the count is that of M A.
* With M = A^{-1} one step solves the system.
* For a fixed linear SPD preconditioner, r_{j+1}.z_j = 0, so the flexible
  (Polak-Ribiere) beta equals the standard one and both give the same iterates.
* For a preconditioner that changes between iterations, the loss of
  conjugacy between consecutive directions follows in closed form from the
  recurrences, and differs between the two betas.
"""
import numpy as np
import pytest

from oracle import pcg


def _spd_with_spectrum(eigs, seed):
    rng = np.random.default_rng(seed)
    n = len(eigs)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.asarray(eigs, dtype=np.float64)) @ Q.T


def _mv(A):
    return lambda X: A @ X


def test_iterates_are_the_krylov_galerkin_projection():
    rng = np.random.default_rng(3)
    n = 40
    A = _spd_with_spectrum(np.linspace(1.0, 50.0, n) ** 1.3, seed=4)
    f = rng.standard_normal(n)
    x_star = np.linalg.solve(A, f)
    prev = np.inf
    for j in range(1, 9):
        u, it, _ = pcg.pcg(_mv(A), None, f, tol=0.0, maxit=j)
        assert it == j
        K = np.empty((n, j))
        v = f.copy()
        for i in range(j):
            K[:, i] = v
            v = A @ v
        V, _ = np.linalg.qr(K)
        x_j = V @ np.linalg.solve(V.T @ A @ V, V.T @ f)
        assert np.linalg.norm(u - x_j) <= 1e-9 * np.linalg.norm(x_j)
        err = np.sqrt((u - x_star) @ A @ (u - x_star))
        assert err < prev
        prev = err


@pytest.mark.parametrize("k", [1, 3, 5])
def test_finite_termination_at_the_number_of_distinct_eigenvalues(k):
    n = 48
    levels = np.linspace(1.0, 9.0, k)
    A = _spd_with_spectrum(np.repeat(levels, n // k + 1)[:n], seed=k)
    f = np.random.default_rng(10 + k).standard_normal(n)
    _, it, rr = pcg.pcg(_mv(A), None, f, tol=1e-11, maxit=50)
    assert it == k and rr <= 1e-11
    if k > 1:
        _, _, rr_short = pcg.pcg(_mv(A), None, f, tol=0.0, maxit=k - 1)
        assert rr_short > 1e-6


def test_preconditioned_termination_follows_the_spectrum_of_MA():
    rng = np.random.default_rng(21)
    n = 36
    C = np.tril(rng.standard_normal((n, n))) + n * np.eye(n)   # M = C C^T, SPD
    B = _spd_with_spectrum(np.repeat([2.0, 5.0, 11.0], n // 3), seed=22)
    Ci = np.linalg.inv(C)
    A = Ci.T @ B @ Ci          # C^T A C = B has three distinct eigenvalues
    A = 0.5 * (A + A.T)
    M = C @ C.T
    f = rng.standard_normal(n)
    u, it, rr = pcg.pcg(_mv(A), lambda X: M @ X, f, tol=1e-10, maxit=50)
    assert it == 3 and rr <= 1e-10
    assert np.linalg.norm(A @ u - f) <= 1e-9 * np.linalg.norm(f)
    _, it_plain, _ = pcg.pcg(_mv(A), None, f, tol=1e-10, maxit=200)
    assert it_plain > 3


def test_exact_preconditioner_solves_in_one_step():
    A = _spd_with_spectrum(np.geomspace(1e-2, 1e2, 30), seed=5)
    Ai = np.linalg.inv(A)
    f = np.random.default_rng(6).standard_normal((30, 3))
    U, its, rr = pcg.pcg(_mv(A), lambda X: Ai @ X, f, tol=1e-10, maxit=10)
    assert np.all(its == 1) and np.all(rr <= 1e-10)
    assert np.allclose(U, np.linalg.solve(A, f), rtol=0, atol=1e-10 * np.abs(np.linalg.solve(A, f)).max())


def test_flexible_beta_equals_standard_for_a_fixed_preconditioner():
    rng = np.random.default_rng(8)
    n = 50
    A = _spd_with_spectrum(np.linspace(1.0, 400.0, n), seed=9)
    D = np.diag(1.0 / np.diag(A))
    f = rng.standard_normal(n)
    for j in (1, 4, 9, 15):
        u_s, _, _ = pcg.pcg(_mv(A), lambda X: D @ X, f, tol=0.0, maxit=j)
        u_f, _, _ = pcg.pcg(_mv(A), lambda X: D @ X, f, tol=0.0, maxit=j, flexible=True)
        assert np.linalg.norm(u_f - u_s) <= 1e-8 * np.linalg.norm(u_s)


def test_zero_right_hand_side_column_is_left_alone():
    A = _spd_with_spectrum(np.linspace(1.0, 4.0, 12), seed=1)
    F = np.random.default_rng(2).standard_normal((12, 3))
    F[:, 1] = 0.0
    U, its, rr = pcg.pcg(_mv(A), None, F, tol=1e-12, maxit=100)
    assert its[1] == 0 and rr[1] == 0.0 and not U[:, 1].any()
    assert np.allclose(U[:, [0, 2]], np.linalg.solve(A, F[:, [0, 2]]), atol=1e-10)


def _variable_diag_precond(d0, d1):
    """z = diag(d_{c mod 2}) r on the c-th call of one solve (a preconditioner
    that changes between iterations, as an inexact inner solve does)."""
    calls = [0]

    def apply(X):
        d = d0 if calls[0] % 2 == 0 else d1
        calls[0] += 1
        return d[:, None] * X
    return apply


@pytest.mark.parametrize("flexible", [False, True])
def test_conjugacy_defect_with_a_variable_preconditioner(flexible):
    """With x_{i+1} = x_i + alpha_i p_i, r_{i+1} = r_i - alpha_i A p_i and
    p_i.A p_i = r_i.z_i / alpha_i, the next direction p_{i+1} = z_{i+1} + beta_i p_i
    has p_{i+1}.A p_i = (z_{i+1}.r_i - z_{i+1}.r_{i+1} + beta_i r_i.z_i) / alpha_i:
    z_{i+1}.r_i / alpha_i for the standard beta and
    (z_{i+1}.r_i - r_{i+1}.z_i) / alpha_i for the flexible one.  Both sides are
    rebuilt here from the iterates alone: alpha_i p_i = x_{i+1} - x_i."""
    rng = np.random.default_rng(31)
    n = 40
    A = _spd_with_spectrum(np.linspace(1.0, 300.0, n), seed=32)
    f = rng.standard_normal(n)
    d0 = 1.0 / np.diag(A)
    d1 = d0 * rng.uniform(0.3, 3.0, n)

    def iterate(t):
        if t == 0:
            return np.zeros(n)
        return pcg.pcg(_mv(A), _variable_diag_precond(d0, d1), f, tol=0.0, maxit=t, flexible=flexible)[0]

    x = [iterate(t) for t in range(7)]
    r = [f - A @ xi for xi in x]
    z = [(d0 if i % 2 == 0 else d1) * r[i] for i in range(7)]
    seen = []
    for i in range(5):
        dx, dx1 = x[i + 1] - x[i], x[i + 2] - x[i + 1]
        a_i = (dx @ A @ dx) / (r[i] @ z[i])
        a_i1 = (dx1 @ A @ dx1) / (r[i + 1] @ z[i + 1])
        lhs = (dx1 / a_i1) @ A @ (dx / a_i)
        rhs = (z[i + 1] @ r[i] - (r[i + 1] @ z[i] if flexible else 0.0)) / a_i
        scale = np.linalg.norm(dx1 / a_i1) * np.linalg.norm(A @ dx / a_i)
        assert abs(lhs - rhs) <= 1e-8 * scale, (i, lhs, rhs, scale)
        seen.append(abs(rhs) / scale)
    assert max(seen) > 1e-4     # the preconditioner change is visible
