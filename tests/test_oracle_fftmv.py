"""Pins of the oracle's FFT product with A (Section 5) against the dense definition."""
import numpy as np
import pytest

import synth
from oracle import cmatvec, fftmv, ie


@pytest.mark.parametrize("d,n", [(2, 16), (2, 33), (2, 64), (3, 8), (3, 11)])
def test_fft_matvec_equals_dense_product(d, n):
    b = synth.coef_smooth(d, n)
    prob = ie.Problem(d, n, b=b, c=b)
    X = synth.rhs(prob.N, 3, seed=5).T.copy()
    ref = prob.dense() @ X
    got = fftmv.FFTMatvec(prob)(X)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # the plain C loop of the oracle agrees as well (two independent definitions)
    assert np.abs(cmatvec.matvec(prob, X) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_fft_matvec_single_vector_and_unequal_coefficients():
    n = 24
    rng = np.random.default_rng(2)
    b, c = 1.0 + 0.3 * rng.random(n * n), 1.0 + 0.3 * rng.random(n * n)
    prob = ie.Problem(2, n, b=b, c=c)
    x = synth.rhs(prob.N, 1, seed=9)[0]
    ref = prob.dense() @ x
    got = fftmv.FFTMatvec(prob)(x)
    assert got.shape == x.shape
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
