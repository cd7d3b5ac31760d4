"""Oracle pins against the paper's printed tables and theorems (Sections 2-5)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import dd, ie, pcg, precond

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
GRID = {"node": ie.GRID_NODE, "cell": ie.GRID_CELL}


def _eig(prob, part, A):
    P = precond.ExactPreconditioner(prob, part, A)
    return precond.preconditioned_eigenvalues(A, P.dense(prob.N))


def _check(ev, pair, tol=1.5e-4):
    assert ev.max() == pytest.approx(pair[0], abs=tol)
    assert ev.min() == pytest.approx(pair[1], abs=tol)


@pytest.mark.parametrize("tab", ["t_cbd_2d", "t_cbd_3d"])
def test_table_cbd(tab):
    g = GOLD[tab]
    for row in g["rows"]:
        n = row["n"]
        d = 2 if tab.endswith("2d") else 3
        prob = ie.Problem(d, n, grid=GRID[g["grid"]])
        A = prob.dense()
        # D = 2^d: Jacobi and Schwarz with m = 2; CBD with m = cbd_m
        _check(_eig(prob, dd.Partition(d, n, 2, 1, dd.JACOBI), A), row["jacobi"])
        _check(_eig(prob, dd.Partition(d, n, 2, 1, dd.SCHWARZ), A), row["schwarz"])
        _check(_eig(prob, dd.Partition(d, n, row["cbd_m"], 1, dd.CBD), A), row["cbd"])


@pytest.mark.parametrize("tab", ["t_schwarz_2d", "t_schwarz_3d"])
def test_table_schwarz(tab):
    g = GOLD[tab]
    d = 2 if tab.endswith("2d") else 3
    for row in g["rows"]:
        prob = ie.Problem(d, row["n"], grid=GRID[g["grid"]])
        A = prob.dense()
        _check(_eig(prob, dd.Partition(d, row["n"], row["m"], 1, dd.JACOBI), A), row["jacobi"])
        _check(_eig(prob, dd.Partition(d, row["n"], row["m"], 1, dd.SCHWARZ), A), row["schwarz"])


def test_table_interface_size():
    g = GOLD["t_d"]
    prob = ie.Problem(2, g["n"], grid=GRID[g["grid"]])
    A = prob.dense()
    L = np.linalg.cholesky(A)
    for row in g["rows"]:
        part = dd.Partition(2, g["n"], g["m"], row["delta"], dd.CBD)
        Minv = precond.ExactPreconditioner(prob, part, A).dense(prob.N)
        S = L.T @ Minv @ L
        lmin = scipy.linalg.eigh(0.5 * (S + S.T), eigvals_only=True, subset_by_index=[0, 0])[0]
        assert lmin == pytest.approx(row["lmin"], abs=1.5e-4)


@pytest.mark.parametrize("d,n,m,mode,mult", [
    (2, 16, 2, dd.SCHWARZ, 4),     # th:max48: lambda_max = 2^d, eigenspace dimension 2^d
    (2, 16, 4, dd.CBD, 36),        # CBD theorem: dimension (2(m-1))^d
    (2, 16, 8, dd.CBD, 196),
    (3, 8, 4, dd.CBD, 216),
])
def test_lambda_max_multiplicity(d, n, m, mode, mult):
    prob = ie.Problem(d, n)
    A = prob.dense()
    ev = _eig(prob, dd.Partition(d, n, m, 1, mode), A)
    top = 2 ** d
    assert ev.max() == pytest.approx(top, abs=1e-9)
    assert np.sum(np.abs(ev - top) < 1e-8) == mult


def test_jacobi_two_block_spectrum_pairs():
    # th:jacobi: with two blocks, the spectrum of T^{-1}A is symmetric about 1
    n = 12
    prob = ie.Problem(2, n)
    A = prob.dense()
    half = np.arange(prob.N) < prob.N // 2
    Minv = np.zeros_like(A)
    for sel in (half, ~half):
        idx = np.nonzero(sel)[0]
        Minv[np.ix_(idx, idx)] = np.linalg.inv(A[np.ix_(idx, idx)])
    ev = np.sort(precond.preconditioned_eigenvalues(A, Minv))
    assert np.allclose(ev, np.sort(2.0 - ev), atol=1e-11)


def test_subdomain_projection_is_identity_on_its_support():
    # l:subdomain: P_i = R_i^T A_i^{-1} R_i A fixes vectors supported in Omega_i
    n = 16
    prob = ie.Problem(2, n)
    A = prob.dense()
    part = dd.Partition(2, n, 4, 1, dd.CBD)
    rng = np.random.default_rng(7)
    for sd in part.subdomains:
        x = np.zeros(prob.N)
        x[sd.index] = rng.standard_normal(len(sd.index))
        Ai = A[np.ix_(sd.index, sd.index)]
        Px = np.zeros(prob.N)
        Px[sd.index] = np.linalg.solve(Ai, (A @ x)[sd.index])
        assert np.allclose(Px, x, atol=1e-10 * np.abs(x).max())


def test_lambda_max_bounded_by_D():
    # th:max: lambda_max(T^{-1}A) <= D for any decomposition
    n = 16
    prob = ie.Problem(2, n)
    A = prob.dense()
    for mode, m in [(dd.JACOBI, 4), (dd.SCHWARZ, 4), (dd.CBD, 4)]:
        part = dd.Partition(2, n, m, 1, mode)
        assert _eig(prob, part, A).max() <= part.D + 1e-9


@pytest.mark.parametrize("row", GOLD["t_it_m48_2d"]["rows"], ids=lambda r: "n%d" % r["n"])
def test_pcg_iterations_exact_subsolves(row):
    n = row["n"]
    prob = ie.Problem(2, n)
    A = prob.dense()
    f = synth.rhs(prob.N, 1, seed=0)[0]
    for key, mode, m in [("jacobi", dd.JACOBI, 2), ("schwarz", dd.SCHWARZ, 2), ("cbd", dd.CBD, n // 4)]:
        P = precond.ExactPreconditioner(prob, dd.Partition(2, n, m, 1, mode), A)
        u, it, rr = pcg.pcg(lambda X: A @ X, P.apply, f, tol=1e-12, maxit=400)
        assert rr <= 1e-12
        assert abs(it - row[key]) <= 2, (key, it, row[key])


@pytest.mark.parametrize("row", GOLD["t_it_m48_3d"]["rows"], ids=lambda r: "n%d" % r["n"])
def test_pcg_iterations_exact_subsolves_3d(row):
    # 3D half of t:it_m48 (cell-centred grid).  CBD partitions are 4 points wide per
    # axis (the reading recorded with the table entry)
    n = row["n"]
    prob = ie.Problem(3, n)
    A = prob.dense()
    f = synth.rhs(prob.N, 1, seed=0)[0]
    w = GOLD["t_it_m48_3d"]["cbd_points_per_partition_axis"]
    for key, mode, m in [("jacobi", dd.JACOBI, 2), ("schwarz", dd.SCHWARZ, 2), ("cbd", dd.CBD, n // w)]:
        P = precond.ExactPreconditioner(prob, dd.Partition(3, n, m, 1, mode), A)
        u, it, rr = pcg.pcg(lambda X: A @ X, P.apply, f, tol=1e-12, maxit=400)
        assert rr <= 1e-12
        assert abs(it - row[key]) <= 2, (key, it, row[key])
