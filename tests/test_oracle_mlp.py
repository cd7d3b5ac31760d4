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


def test_adam_first_step_and_gradient_scale_invariance():
    """Two properties of Adam (Kingma and Ba, Section 2.1) that do not restate its
    update: the bias-corrected first step moves each parameter by lr * |g| / (|g| + eps)
    against the sign of g, the step size lr when |g| >> eps and less when |g| is
    near eps; and rescaling every gradient by c > 0 leaves the trajectory unchanged
    while |g| >> eps."""
    lr, eps = 1e-2, 1e-8
    g = np.array([3.0, -0.5, 1e-4, -1e-6, 2e-8, 0.0])
    p0 = np.zeros_like(g)
    p1, m, v = mlp.adam(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    step = -(p1 - p0)
    assert np.allclose(step, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    assert abs(step[3]) > 0.98 * lr and abs(step[4]) < 0.7 * lr and step[5] == 0.0

    rng = np.random.default_rng(4)
    gs = rng.standard_normal((12, 8)) * rng.uniform(0.5, 2.0, (12, 1))
    traj = []
    for c in (1.0, 1e3):
        p, m, v = np.zeros(8), np.zeros(8), np.zeros(8)
        for s, gt in enumerate(gs, start=1):
            p, m, v = mlp.adam(p, c * gt, m, v, s, lr)
        traj.append(p)
    assert np.allclose(traj[0], traj[1], rtol=1e-6, atol=1e-9)
