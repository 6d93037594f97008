"""Pins of the FP64 network reference (CPU): the analytic gradient against
central finite differences of the loss, and Adam against its definition on a
quadratic with a known minimiser."""
import numpy as np

from oracle import mlp_ref


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    C = 4
    theta = rng.normal(0, 0.2, mlp_ref.n_params(C))
    X = rng.dirichlet(np.ones(256), size=5)
    T = rng.uniform(0, 1, (5, C))
    g = mlp_ref.grad(theta, X, T, C)
    idx = rng.choice(theta.size, 300, replace=False)
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp_ref.loss(tp, X, T, C) - mlp_ref.loss(tm, X, T, C)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_layout_and_size():
    assert mlp_ref.n_params(4) == 256 * 128 + 128 + 128 * 64 + 64 + 64 * 4 + 4 == 41412


def test_adam_converges_on_quadratic():
    theta = np.array([3.0, -2.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for step in range(1, 5001):
        g = 2 * (theta - np.array([0.5, 1.5]))
        theta, m, v = mlp_ref.adam_step(theta, g, m, v, step, lr=1e-2)
    assert np.max(np.abs(theta - [0.5, 1.5])) < 1e-3


def test_adam_first_step_is_sign_times_lr():
    """With bias correction the first Adam step moves each parameter by lr in
    the direction opposite the gradient's sign (for |g| >> eps)."""
    theta = np.array([1.0, 1.0, 1.0])
    g = np.array([0.3, -2.0, 5e-3])
    t, _, _ = mlp_ref.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(t, theta - 0.01 * np.sign(g), atol=1e-7)
