"""Pins of the rank-predictor oracle: gradient by finite differences, bf16 rounding, Adam."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_rule():
    x = np.array([1.0, 1.00390625, 1.0078125, 1.01171875, -3.0, 0.0], dtype=np.float32)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    # 1 + 3*2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert list(mlp.bf16_round(x)) == [1.0, 1.0, 1.0078125, 1.015625, -3.0, 0.0]
    y = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    r = mlp.bf16_round(y)
    assert np.all(np.abs(r - y) <= np.abs(y) * 2.0 ** -8)
    assert np.all(r.view(np.uint32) & 0xFFFF == 0)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(3).astype(np.float64)
    X = rng.standard_normal((40, mlp.F))
    t = rng.standard_normal(40)
    loss, g = mlp.loss_and_grad(p, X, t, rounded=False)
    idx = rng.choice(len(p), 60, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = 1e-6
        lp, _ = mlp.loss_and_grad(p + e, X, t, rounded=False)
        lm, _ = mlp.loss_and_grad(p - e, X, t, rounded=False)
        fd = (lp - lm) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_reduces_a_quadratic_and_fits_a_line():
    # a network trained by the oracle's own Adam fits a smooth target
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (200, mlp.F))
    t = 2.0 * X[:, 0] - X[:, 1] + 0.5
    p = mlp.init_params(0).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0, _ = mlp.loss_and_grad(p, X, t)
    for s in range(1, 301):
        loss, g = mlp.loss_and_grad(p, X, t)
        p, m, v = mlp.adam(p, g, m, v, s, 1e-2)
    assert loss < 0.02 * l0
