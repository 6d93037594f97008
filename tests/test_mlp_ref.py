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


def test_bf16_round_matches_the_format():
    """Values fixed by the bfloat16 format: 8 significant bits, ties to even."""
    r = mlp_ref.bf16_round
    assert r(1.0) == 1.0
    assert r(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7            # representable
    assert r(1.0 + 2.0 ** -8) == 1.0                        # tie, 1.0 is even
    assert r(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6        # tie, rounds to the even neighbour above
    assert r(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert r(-(1.0 + 2.0 ** -8 + 2.0 ** -20)) == -(1.0 + 2.0 ** -7)
    assert r(0.0) == 0.0
    assert r(3.0) == 3.0 and r(255.0) == 255.0 and r(257.0) == 256.0 and r(259.0) == 260.0
    # against the bit-level definition on random FP32 values: keep the top 16
    # bits after adding 0x7FFF plus the lowest kept bit
    rng = np.random.default_rng(0)
    f = (rng.standard_normal(10000) * 10.0 ** rng.uniform(-6, 6, 10000)).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    want = u.astype(np.uint32).view(np.float32).astype(np.float64)
    assert np.array_equal(r(f.astype(np.float64)), want)


def test_forward_bf16_reduces_to_forward_on_representable_values():
    """With parameters and inputs already BF16 values and exact products, the
    BF16 forward equals the FP64 one up to the hidden-layer roundings; with
    tiny-magnitude hidden activations that are BF16 values it is identical."""
    C = 3
    theta = np.zeros(mlp_ref.n_params(C))
    W1, b1, W2, b2, W3, b3 = mlp_ref.unpack(theta, C)
    W1[0, 0] = 1.0
    W2[0, 0] = 0.5
    W3[0, :] = [1.0, 2.0, -0.25]
    b3[:] = [0.125, 0.0, 1.0]
    X = np.zeros((2, 256))
    X[0, 0] = 0.375
    X[1, 0] = 0.75
    assert np.array_equal(mlp_ref.forward_bf16(theta, X, C), mlp_ref.forward(theta, X, C)[0])
