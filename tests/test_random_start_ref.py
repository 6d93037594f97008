"""Pins of the paper's own start (random memberships, centroids first) in the
oracle, and of the counter generator its random weights come from."""
import numpy as np
import pytest

from oracle import fcm_ref
from phantom import counter_u64, uniform24


def test_counter_generator_is_splitmix64():
    """Draws 0, 1, 2 of the stream with state 0 are the first three outputs of
    SplitMix64 seeded with 0 (the published reference values)."""
    got = counter_u64(0, np.arange(3, dtype=np.uint64))
    assert [int(v) for v in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform24_exact_in_fp32():
    r = uniform24(12345, np.arange(100000, dtype=np.uint64))
    assert np.all(r > 0.0) and np.all(r <= 1.0)
    assert np.array_equal(r.astype(np.float32).astype(np.float64), r)
    k = r * 2.0 ** 24
    assert np.array_equal(k, np.rint(k))
    # top 24 bits of the draw, plus one
    h = counter_u64(12345, np.arange(10, dtype=np.uint64))
    assert np.array_equal(r[:10], ((h >> np.uint64(40)).astype(np.float64) + 1) / 2.0 ** 24)


def test_two_voxel_example_by_hand():
    """x = {0, 10}, C = 2, m = 2, U^0 rows (3/4, 1/4) and (1/4, 3/4) (from
    weights 3:1 and 1:3).  Eq.3 with u^2 weights: v^1 = (0.0625*10 / 0.625,
    0.5625*10 / 0.625) = (1, 9).  Eq.4 at v^1: voxel 0 is at distances 1 and 9,
    u = (81/82, 1/82); voxel 10 mirrored.  delta^1 = 81/82 - 3/4.
    J^1 = 2 (6561 + 81) / 6724.  v^2_0 = (1/82)^2 10 / ((81/82)^2 + (1/82)^2)
    = 10/6562."""
    x = np.array([0, 10], np.uint8)
    r = np.array([[3.0, 1.0], [1.0, 3.0]])
    tr = fcm_ref.solve_random_u(x, 2, 2.0, 0.0, 2, r)
    assert np.all(np.isnan(tr.v[0])) and np.isnan(tr.delta[0]) and np.isnan(tr.J[0])
    assert np.allclose(tr.v[1], [1.0, 9.0], rtol=0, atol=1e-13)
    assert tr.delta[1] == pytest.approx(81 / 82 - 3 / 4, abs=1e-15)
    assert tr.J[1] == pytest.approx(2 * 6642 / 6724, rel=1e-14)
    assert np.allclose(tr.v[2], [10 / 6562, 10 - 10 / 6562], rtol=0, atol=1e-12)


def test_fuzziness_weights_memberships():
    """Same U^0 with m = 3: v^1_0 = (1/64) 10 / (28/64) = 5/14, v^1_1 = 135/14
    (the weights are u^m, not u)."""
    tr = fcm_ref.solve_random_u(np.array([0, 10], np.uint8), 2, 3.0, 0.0, 1,
                                np.array([[3.0, 1.0], [1.0, 3.0]]))
    assert np.allclose(tr.v[1], [5 / 14, 135 / 14], rtol=1e-14)


@pytest.mark.parametrize("m", [1.5, 2.0, 2.5])
def test_uniform_start_closed_form(m):
    """Equal weights: every u^0 = 1/C, so every v^1 is the data mean; at
    centroids that coincide every membership is 1/C again, so delta^1 = 0, the
    solve stops at T = 1 with v^T = mean, and J^1 = C^(1 - m) sum (x - mean)^2."""
    rng = np.random.default_rng(4)
    x = rng.integers(0, 256, 999).astype(np.uint8)
    C = 4
    tr = fcm_ref.solve_random_u(x, C, m, 0.005, 50, np.ones((x.size, C)))
    mean = x.astype(np.float64).mean()
    assert tr.T == 1 and tr.status == fcm_ref.OK
    assert np.allclose(tr.v[1], mean, rtol=1e-13)
    assert tr.delta[1] == pytest.approx(0.0, abs=1e-15)
    assert tr.J[1] == pytest.approx(C ** (1 - m) * np.sum((x - mean) ** 2), rel=1e-12)


def test_continues_as_centroid_first_after_first_update():
    """From v^1 on, the iteration is the centroid-first one started at v^1:
    same centroids and objective, and the same changes from t = 2 on (delta^1
    alone compares with the random U^0)."""
    rng = np.random.default_rng(9)
    x = rng.integers(0, 256, 3000).astype(np.uint8)
    r = uniform24(77, np.arange(3000 * 3, dtype=np.uint64)).reshape(3000, 3)
    tr = fcm_ref.solve_random_u(x, 3, 2.0, 0.0, 12, r)
    cf = fcm_ref.solve(x, 3, 2.0, 0.0, 11, v0=tr.v[1])
    for t in range(1, 13):
        assert np.allclose(tr.v[t], cf.v[t - 1], rtol=1e-13, atol=1e-12)
        assert tr.J[t] == pytest.approx(cf.J[t - 1], rel=1e-12)
        if t >= 2:
            assert tr.delta[t] == pytest.approx(cf.delta[t - 1], abs=1e-14)
    assert tr.delta[1] > 0.05  # the random U^0 is far from any fixed point
