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


def _hand_network():
    """A network with a handful of nonzero parameters whose outputs are worked
    out by hand below: nonzero hidden biases, one negative pre-activation in
    each hidden layer for one of the two samples, and a unit fed only by its
    bias.  Every value is a short dyadic fraction, exact in FP64 and in BF16."""
    C = 2
    theta = np.zeros(mlp_ref.n_params(C))
    W1, b1, W2, b2, W3, b3 = mlp_ref.unpack(theta, C)
    # layer 1: z1_0 = x0 + 2 x1 + 1/2, z1_1 = -3 x0 + 1, z1_2 = 4 x1 - 1,
    # z1_3 = -1/4 (always cut by the ReLU), z1_4 = 3/4 (bias only)
    W1[0, 0], W1[1, 0], b1[0] = 1.0, 2.0, 0.5
    W1[0, 1], b1[1] = -3.0, 1.0
    W1[1, 2], b1[2] = 4.0, -1.0
    b1[3] = -0.25
    b1[4] = 0.75
    # layer 2: z2_0 = h0 - 2 h1 + h2/2 + h4 + 1/4, z2_1 = -h0 + 2 h2 - 1/2
    W2[0, 0], W2[1, 0], W2[2, 0], W2[4, 0], b2[0] = 1.0, -2.0, 0.5, 1.0, 0.25
    W2[0, 1], W2[2, 1], b2[1] = -1.0, 2.0, -0.5
    # output: y0 = 2 g0 + g1 - 1, y1 = -g0 + 4 g1 + 1/2
    W3[0, 0], W3[1, 0], b3[0] = 2.0, 1.0, -1.0
    W3[0, 1], W3[1, 1], b3[1] = -1.0, 4.0, 0.5
    X = np.zeros((2, 256))
    X[0, :2] = [0.5, 0.25]
    X[1, :2] = [0.125, 0.75]
    return theta, X, C


def test_forward_fixed_values_worked_by_hand():
    """Sample A (x0 = 1/2, x1 = 1/4):
      z1 = (3/2, -1/2, 0, -1/4, 3/4) -> h1 = (3/2, 0, 0, 0, 3/4)   (z1_1 < 0 cut)
      z2 = (3/2 + 3/4 + 1/4, -3/2 - 1/2) = (5/2, -2) -> h2 = (5/2, 0)   (z2_1 < 0 cut)
      y  = (5 - 1, -5/2 + 1/2) = (4, -2)                              (no ReLU on y)
    Sample B (x0 = 1/8, x1 = 3/4):
      z1 = (17/8, 5/8, 2, -1/4, 3/4) -> h1 = (17/8, 5/8, 2, 0, 3/4)
      z2 = (17/8 - 5/4 + 1 + 3/4 + 1/4, -17/8 + 4 - 1/2) = (23/8, 11/8)
      y  = (23/4 + 11/8 - 1, -23/8 + 11/2 + 1/2) = (49/8, 25/8)
    A dropped hidden bias, a ReLU missing from either hidden layer, a ReLU on
    the output or a transposed layer each change at least one of these."""
    theta, X, C = _hand_network()
    y, (_, z1, h1, z2, h2) = mlp_ref.forward(theta, X, C)
    assert z1[0, :5].tolist() == [1.5, -0.5, 0.0, -0.25, 0.75]
    assert h1[1, :5].tolist() == [2.125, 0.625, 2.0, 0.0, 0.75]
    assert z2[:, :2].tolist() == [[2.5, -2.0], [2.875, 1.375]]
    assert h2[0, :2].tolist() == [2.5, 0.0]
    assert y.tolist() == [[4.0, -2.0], [6.125, 3.125]]
    # every value above is a BF16 value, so the BF16 forward is exact too
    assert mlp_ref.forward_bf16(theta, X, C).tolist() == [[4.0, -2.0], [6.125, 3.125]]


def test_gradient_fixed_values_worked_by_hand():
    """The chain rule on the hand network with targets t = y - (1, 0) for
    sample A and t = y for sample B: dL/dy = 2 (y - t) / (B C) = (1/2, 0) on
    sample A only.  Then dL/db3 = (1/2, 0), dL/dW3[0,0] = g0(A)/2 = 5/4,
    dL/dW3[1,0] = g1(A)/2 = 0, and back through the active units of sample A:
    dL/dz2_0 = 2 * 1/2 = 1 (z2_1 was cut), dL/db2 = (1, 0),
    dL/dW2[0,0] = h0 = 3/2, dL/dW2[4,0] = h4 = 3/4, dL/dW2[1,0] = h1 = 0;
    dL/dz1 = W2[:, 0] masked by z1 > 0 = (1, 0, 0, 0, 1), so
    dL/db1[:5] = (1, 0, 0, 0, 1), dL/dW1[0,0] = x0 = 1/2, dL/dW1[1,0] = 1/4."""
    theta, X, C = _hand_network()
    y, _ = mlp_ref.forward(theta, X, C)
    T = y.copy()
    T[0, 0] -= 1.0
    g = mlp_ref.unpack(mlp_ref.grad(theta, X, T, C), C)
    gW1, gb1, gW2, gb2, gW3, gb3 = g
    assert gb3.tolist() == [0.5, 0.0]
    assert gW3[:2].tolist() == [[1.25, 0.0], [0.0, 0.0]]
    assert gb2[:2].tolist() == [1.0, 0.0]
    assert [gW2[0, 0], gW2[1, 0], gW2[4, 0], gW2[2, 0]] == [1.5, 0.0, 0.75, 0.0]
    assert gb1[:5].tolist() == [1.0, 0.0, 0.0, 0.0, 1.0]
    assert [gW1[0, 0], gW1[1, 0], gW1[0, 4]] == [0.5, 0.25, 0.5]
    assert np.count_nonzero(gW1) == 4      # W1[0,0], W1[1,0], W1[0,4], W1[1,4]
