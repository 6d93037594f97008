"""Oracle-F (C, threaded) against the literal numpy oracle: every step of the
trajectory agrees to within what FP64 summation order allows (centroids and
J to 1e-11 relative, the change to 1e-10), the same iteration count, for
several thread counts, cluster counts, fuzziness values and the
zero-distance cases.  The sums over the voxels are added in another order
(chunks per thread), which moves the centroids by ~1e-13 relative; early
iterations can amplify that by the step's Jacobian, and the change reacts
to a centroid difference with the sensitivity of Eq.4."""
import numpy as np
import pytest

from oracle import fcm_fast, fcm_ref
from phantom import PhantomParams, phantom, phantom_2d


def same(a, b, tol=1e-11, dtol=1e-10):
    assert a.T == b.T and a.status == b.status
    for t in range(a.T + 1):
        assert np.allclose(a.v[t], b.v[t], rtol=tol, atol=tol), (t, a.v[t], b.v[t])
        assert abs(a.J[t] - b.J[t]) <= tol * max(abs(b.J[t]), 1.0), (t, a.J[t], b.J[t])
        if t > 0:
            assert abs(a.delta[t] - b.delta[t]) <= dtol, (t, a.delta[t], b.delta[t])


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_slice_config1(threads):
    x = phantom_2d(200, 200, seed=1)
    same(fcm_fast.solve(x, 4, threads=threads), fcm_ref.solve(x, 4))


@pytest.mark.parametrize("C,m", [(2, 2.0), (8, 2.0), (4, 1.5), (5, 2.5), (3, 3.0)])
def test_clusters_and_fuzziness(C, m):
    x = phantom(PhantomParams(shape=(12, 64, 64), seed=4 + C))
    same(fcm_fast.solve(x, C, m=m, eps=1e-6, threads=4), fcm_ref.solve(x, C, m=m, eps=1e-6))


def test_given_start_and_max_iter():
    x = phantom_2d(90, 110, seed=6)
    v0 = np.array([3.0, 55.5, 120.0, 180.0])
    same(fcm_fast.solve(x, 4, v0=v0, max_iter=4, eps=1e-12), fcm_ref.solve(x, 4, v0=v0, max_iter=4, eps=1e-12))


@pytest.mark.parametrize("case", ["constant", "two_levels", "on_level"])
def test_zero_distance(case):
    rng = np.random.default_rng(2)
    if case == "constant":
        x, C, v0 = np.full(500, 77, np.uint8), 3, None
    elif case == "two_levels":
        x, C, v0 = np.where(rng.random(700) < 0.3, 20, 200).astype(np.uint8), 2, None
    else:
        x, C, v0 = rng.integers(0, 256, 999).astype(np.uint8), 4, np.array([0.0, 64.0, 128.0, 255.0])
    same(fcm_fast.solve(x, C, v0=v0, threads=2), fcm_ref.solve(x, C, v0=v0))


def test_thread_counts_agree_on_a_volume():
    x = phantom(PhantomParams(shape=(40, 96, 96), seed=3))
    a = fcm_fast.solve(x, 4, threads=1)
    for p in (2, 5, 16):
        same(fcm_fast.solve(x, 4, threads=p), a)
