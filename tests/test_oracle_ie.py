"""Pins of the oracle's discretization (Section 2.1) against quadrature and exact relations."""
import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import ie, cmatvec


@pytest.mark.parametrize("h", [1 / 8, 1 / 64, 1 / 512])
def test_self_cell_2d_matches_quadrature(h):
    a = h / 2
    f = lambda y, x: -np.log(x * x + y * y) / (4 * np.pi)
    # the integrand is symmetric under the 8 symmetries of the square
    v, _ = integrate.dblquad(f, 0, a, lambda x: 0, lambda x: x, epsabs=0, epsrel=1e-13)
    assert ie.self_cell_integral(2, h) == pytest.approx(8 * v, rel=1e-13)


@pytest.mark.parametrize("h", [1 / 4, 1 / 32])
def test_self_cell_3d_matches_quadrature(h):
    a = h / 2
    f = lambda z, y, x: 1 / (4 * np.pi * np.sqrt(x * x + y * y + z * z))
    v, _ = integrate.tplquad(f, 0, a, lambda x: 0, lambda x: a, lambda x, y: 0, lambda x, y: a,
                             epsabs=0, epsrel=1e-11)
    assert ie.self_cell_integral(3, h) == pytest.approx(8 * v, rel=1e-10)


def test_kernel_values():
    # (e:k): K(1) = 0 in 2D; K(e^{-2 pi}) = 1; 3D K(r) = 1/(4 pi r)
    assert ie.kernel(2, 1.0) == 0.0
    assert ie.kernel(2, np.exp(-2 * np.pi)) == pytest.approx(1.0, rel=1e-15)
    assert ie.kernel(3, 0.5) == pytest.approx(1 / (2 * np.pi), rel=1e-15)


def test_grid_points_order_and_spacing():
    x = ie.grid_points(2, 4)
    assert np.allclose(x[:5], [[0.125, 0.125], [0.375, 0.125], [0.625, 0.125], [0.875, 0.125], [0.125, 0.375]])
    x3 = ie.grid_points(3, 3)
    assert np.allclose(x3[3 * 3 + 3 + 1], [0.5, 0.5, 0.5])
    xn = ie.grid_points(2, 5, ie.GRID_NODE)
    assert np.allclose(xn[6], [0.25, 0.25])


def test_matrix_entry_by_hand():
    p = ie.Problem(2, 4)
    # points 0 and 1 are h apart: A_01 = h^2 * (-(1/2pi) log h)
    h = 0.25
    assert p.block([0], [1])[0, 0] == pytest.approx(-h * h * np.log(h) / (2 * np.pi), rel=1e-15)
    # points 0 and 5 are h*sqrt2 apart
    assert p.block([5], [0])[0, 0] == pytest.approx(-h * h * np.log(h * np.sqrt(2)) / (2 * np.pi), rel=1e-15)
    p3 = ie.Problem(3, 4)
    assert p3.block([0], [16])[0, 0] == pytest.approx(h ** 3 / (4 * np.pi * h), rel=1e-15)


@pytest.mark.parametrize("d,n", [(2, 16), (3, 6)])
def test_symmetric_positive_definite(d, n):
    p = ie.Problem(d, n)
    A = p.dense()
    assert np.array_equal(A, A.T)
    np.linalg.cholesky(A)
    assert np.linalg.eigvalsh(A).min() > 0


def test_condition_number_grows_like_N_in_2d():
    # Section 2.1: cond(A) = O(N) in 2D; doubling n multiplies cond by ~4
    c = [np.linalg.cond(ie.Problem(2, n).dense()) for n in (8, 16, 32)]
    assert 2.5 < c[1] / c[0] < 5.5 and 2.5 < c[2] / c[1] < 5.5


def test_coefficients_scale_rows_and_columns():
    # (e:int) with b = c: A_bc = D A D, so A_bc^{-1} f = D^{-1} A^{-1} D^{-1} f
    n = 12
    b = synth.coef_smooth(2, n)
    p0 = ie.Problem(2, n)
    p1 = ie.Problem(2, n, b=b, c=b)
    f = synth.rhs(p0.N, 1, seed=3)[0]
    u1 = np.linalg.solve(p1.dense(), f)
    u0 = np.linalg.solve(p0.dense(), f / b) / b
    assert np.allclose(u1, u0, rtol=1e-10, atol=0)
    # unequal b, c: entry (i,j) = b_i A_ij c_j
    c = 2.0 - b
    p2 = ie.Problem(2, n, b=b, c=c)
    assert p2.block([3], [7])[0, 0] == pytest.approx(b[3] * p0.block([3], [7])[0, 0] * c[7], rel=1e-15)
    # the diagonal: b_i c_i times the self-cell integral, in 2D and 3D
    assert p2.diag() == pytest.approx(b * c * ie.self_cell_integral(2, 1.0 / n), rel=1e-15)
    q0 = ie.Problem(3, 5)
    b3 = synth.coef_smooth(3, 5)
    q1 = ie.Problem(3, 5, b=b3, c=1.0 / b3)
    assert np.allclose(q1.diag(), np.diag(q1.dense()), rtol=1e-15, atol=0)
    assert np.allclose(q1.diag(), q0.diag(), rtol=1e-14, atol=0)


def test_coef_field_range():
    c = synth.coef_smooth(2, 64)
    assert c.min() >= 0.5 - 1e-15 and c.max() <= 1.5 + 1e-15
    assert c.min() < 0.51 and c.max() > 1.49


@pytest.mark.parametrize("d,n,nrhs", [(2, 24, 1), (2, 17, 5), (3, 7, 3)])
def test_c_matvec_matches_dense(d, n, nrhs):
    b = synth.coef_smooth(d, n)
    p = ie.Problem(d, n, b=b, c=b)
    x = synth.rhs(p.N, nrhs, seed=1).T
    ref = p.dense() @ x
    y = cmatvec.matvec(p, x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    rows = np.array([0, 5, p.N - 1])
    assert np.allclose(cmatvec.matvec(p, x, rows=rows), ref[rows], rtol=1e-13, atol=1e-16)
