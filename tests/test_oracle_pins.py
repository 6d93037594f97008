"""Pins of the FP64 oracle against what the paper and mathematics fix (CPU only).

Each test checks the oracle against something other than itself: exact
rational or high-precision arithmetic, the first-order optimality conditions
of the objective (Eq.1 under the constraint Eq.2), invariants, symmetries,
limits, and the brFCM regrouping.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, fcm_hist, fcm_ref
from phantom import phantom_2d, phantom_3d

RNG = np.random.default_rng(12345)


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1.0))


@pytest.fixture(scope="module")
def img1():
    return phantom_2d(200, 200, seed=1)


# --- exact arithmetic ------------------------------------------------------

@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("case", range(6))
def test_rational_steps(m, case):
    """m = 2, 3: Eq.3/Eq.4 are rational.  Every step of the FP64 trajectory must
    match one exact rational step taken from the same FP64 centroids."""
    rng = np.random.default_rng(100 + case)
    n = int(rng.integers(3, 9))
    C = int(rng.integers(2, 5))
    x = rng.integers(0, 256, n).astype(np.uint8)
    if case == 0:
        x[:] = [0, 0, 10, 11, 200, 201, 255, 128][:n]
    v0 = np.sort(rng.uniform(0, 255, C)).astype(np.float32).astype(np.float64)
    iters = 6
    tr = fcm_ref.solve(x, C, float(m), eps=0.0, max_iter=iters, v0=v0)
    for t in range(iters):
        v1, d1, J1 = exact.step_rational(x, [Fraction(a) for a in tr.v[t]], m)
        assert _rel(tr.v[t + 1], [float(a) for a in v1]) < 1e-13, t
        assert abs(tr.J[t + 1] - float(J1)) <= 1e-12 * max(1.0, float(J1))
        assert abs(tr.delta[t + 1] - float(d1)) <= 1e-13


def test_rational_trajectory_short():
    """Two whole exact iterations from the start (the exact numbers grow ~25x
    in digits per iteration, so longer exact runs are impractical)."""
    x = np.array([0, 0, 10, 11, 200, 201], dtype=np.uint8)
    v0 = [Fraction(1), Fraction(100), Fraction(250)]
    tr = fcm_ref.solve(x, 3, 2.0, eps=0.0, max_iter=2, v0=np.array([1.0, 100.0, 250.0]))
    vs, ds, Js = exact.solve_rational(x, v0, 2, 2)
    for t in range(3):
        assert _rel(tr.v[t], [float(a) for a in vs[t]]) < 1e-14
        assert abs(tr.J[t] - float(Js[t])) <= 1e-13 * float(Js[t])


@pytest.mark.parametrize("m", [1.5, 2.5, 1.25])
def test_decimal_trajectory(m):
    """Any m: a 60-digit decimal run of the same iteration pins the FP64 one."""
    rng = np.random.default_rng(7)
    x = rng.integers(0, 256, 7).astype(np.uint8)
    v0 = np.array([20.0, 120.0, 230.0])
    tr = fcm_ref.solve(x, 3, m, eps=0.0, max_iter=8, v0=v0)
    vs, ds, Js = exact.solve_decimal(x, list(v0), m, 8)
    for t in range(9):
        assert _rel(tr.v[t], [float(a) for a in vs[t]]) < 1e-12
        assert abs(tr.J[t] - float(Js[t])) <= 1e-11 * max(1.0, float(Js[t]))


# --- optimality conditions of Eq.1 under Eq.2 -------------------------------

@pytest.mark.parametrize("m", [1.5, 2.0, 2.5, 3.0])
def test_membership_kkt(img1, m):
    """At fixed v, Eq.4 minimises J over rows on the simplex: the partial
    derivative m u_ij^(m-1) d_ij^2 is the same for every j of a row."""
    x = img1.ravel()[::7]
    v = np.array([3.3, 41.7, 115.1, 162.9])
    U = fcm_ref.memberships(x, v, m)
    g = m * U ** (m - 1) * (x[:, None].astype(np.float64) - v[None, :]) ** 2
    spread = (g.max(axis=1) - g.min(axis=1)) / g.max(axis=1)
    assert np.max(spread) < 1e-12
    assert np.all(U > 0) and np.all(U < 1)


@pytest.mark.parametrize("m", [1.5, 2.0, 2.5])
def test_centroid_stationary(img1, m):
    """At fixed U, Eq.3 zeroes dJ/dv_j = -2 sum_i u_ij^m (x_i - v_j)."""
    x = img1.ravel().astype(np.float64)
    U = fcm_ref.memberships(x, np.array([10.0, 50.0, 100.0, 170.0]), m)
    v = fcm_ref.centroids(x, U, m, np.zeros(4))
    a = U ** m
    grad = (a * (x[:, None] - v[None, :])).sum(axis=0)
    scale = (a * np.abs(x[:, None] - v[None, :])).sum(axis=0)
    assert np.max(np.abs(grad) / scale) < 1e-10


def test_objective_matches_brute_force():
    """Eq.1 evaluated voxel by voxel in exact rationals."""
    x = np.array([0, 5, 9, 200, 201], dtype=np.uint8)
    v = np.array([1.5, 100.25, 199.75])
    U = fcm_ref.memberships(x, v, 2.0)
    brute = sum(Fraction(U[i, j]) ** 2 * (Fraction(int(x[i])) - Fraction(v[j])) ** 2
                for i in range(5) for j in range(3))
    assert abs(fcm_ref.objective(x, U, v, 2.0) - float(brute)) < 1e-12 * float(brute)


# --- invariants --------------------------------------------------------------

@pytest.mark.parametrize("m", [1.5, 2.0, 2.5])
def test_rows_sum_to_one(img1, m):
    U = fcm_ref.memberships(img1, np.array([0.0, 40.0, 110.0, 150.0, 201.5]), m)
    assert np.max(np.abs(U.sum(axis=1) - 1.0)) <= 1e-14
    assert 0.0 < U.sum(axis=0).min() and U.sum(axis=0).max() < U.shape[0]


@pytest.mark.parametrize("m,C", [(2.0, 4), (1.5, 4), (2.5, 4), (2.0, 8), (2.0, 3)])
def test_objective_non_increasing(img1, m, C):
    tr = fcm_ref.solve(img1, C, m, eps=1e-5, max_iter=60)
    J = np.array(tr.J)
    assert np.all(J[1:] <= J[:-1] * (1 + 1e-12))


def test_zero_distance_gets_full_membership():
    x = np.array([0, 7, 100, 255], dtype=np.uint8)
    v = np.array([7.0, 100.0, 180.0])
    U = fcm_ref.memberships(x, v, 2.0)
    assert U[1].tolist() == [1.0, 0.0, 0.0]
    assert U[2].tolist() == [0.0, 1.0, 0.0]
    # two coinciding centroids at the voxel: equal split
    U2 = fcm_ref.memberships(np.array([50], dtype=np.uint8), np.array([50.0, 50.0, 90.0]), 2.0)
    assert U2[0].tolist() == [0.5, 0.5, 0.0]


def test_two_levels_linspace_exact():
    """Two grey levels a < b with C = 2: linspace init puts v at (a, b), T = 1, exact."""
    x = np.array([30] * 50 + [170] * 70, dtype=np.uint8)
    tr = fcm_ref.solve(x, 2, 2.0, 1e-5, 300)
    assert tr.T == 1 and tr.status == fcm_ref.OK
    assert tr.centroids.tolist() == [30.0, 170.0]


@pytest.mark.parametrize("m", [1.5, 2.0, 2.5])
def test_two_levels_converge_to_levels(m):
    x = np.array([30] * 50 + [170] * 70, dtype=np.uint8)
    tr = fcm_ref.solve(x, 2, m, 1e-12, 300, v0=np.array([65.0, 135.0]))
    assert tr.status == fcm_ref.OK
    assert np.max(np.abs(tr.centroids - np.array([30.0, 170.0]))) < 1e-9


def test_linspace_init_values():
    for lo, hi, C in [(0, 255, 4), (0, 193, 3), (3, 197, 8), (17, 17, 4), (0, 1, 8)]:
        v = fcm_ref.linspace_init(lo, hi, C)
        for j in range(C):
            exact_val = Fraction(lo) + Fraction(j * (hi - lo), C - 1)
            assert v[j] == float(np.float32(float(exact_val))), (lo, hi, C, j)
    assert fcm_ref.linspace_init(0, 255, 4).tolist() == [0.0, 85.0, 170.0, 255.0]


# --- symmetries ----------------------------------------------------------------

def test_shift_invariance():
    img = phantom_2d(64, 64, seed=5)
    x = np.minimum(img.astype(np.int32), 200).astype(np.uint8)
    a = fcm_ref.solve(x, 4, 2.0, 1e-5, 300)
    b = fcm_ref.solve((x + 40).astype(np.uint8), 4, 2.0, 1e-5, 300, v0=a.v[0] + 40.0)
    assert a.T == b.T
    assert np.max(np.abs(a.centroids + 40.0 - b.centroids)) < 1e-9
    assert np.array_equal(fcm_ref.defuzzify(x, a.centroids), fcm_ref.defuzzify(x + 40, b.centroids))


def test_permutation_invariance():
    img = phantom_2d(64, 64, seed=6).ravel()
    p = np.random.default_rng(1).permutation(img.size)
    a = fcm_ref.solve(img, 4, 2.0, 1e-5, 300)
    b = fcm_ref.solve(img[p], 4, 2.0, 1e-5, 300)
    assert a.T == b.T and _rel(a.centroids, b.centroids) < 1e-12


def test_symmetric_histogram():
    """Data symmetric about mu with symmetric init keeps v_0 + v_(C-1) = 2 mu."""
    base = np.array([10, 10, 11, 30, 40, 40, 41, 60, 75, 80, 99], dtype=np.int32)
    mu = 120
    x = np.concatenate([mu - base, mu + base]).astype(np.uint8)
    tr = fcm_ref.solve(x, 4, 2.0, 1e-10, 300)
    v = tr.centroids
    assert abs(v[0] + v[3] - 2 * mu) < 1e-9 and abs(v[1] + v[2] - 2 * mu) < 1e-9


# --- limits ----------------------------------------------------------------------

def _lloyd(x, v, iters=100):
    x = x.astype(np.float64)
    for _ in range(iters):
        lab = np.argmin(np.abs(x[:, None] - v[None, :]), axis=1)
        v = np.array([x[lab == k].mean() if np.any(lab == k) else v[k] for k in range(len(v))])
    return v, lab


def test_hard_limit_matches_kmeans():
    """m -> 1 gives hard k-means: with m = 1.05 on well-separated data the
    defuzzified labels equal Lloyd's labels from the same start."""
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.integers(10, 30, 300), rng.integers(100, 120, 300),
                        rng.integers(200, 230, 300)]).astype(np.uint8)
    v0 = np.array([10.0, 120.0, 230.0])
    tr = fcm_ref.solve(x, 3, 1.05, 1e-9, 300, v0=v0)
    vk, lab = _lloyd(x, v0)
    assert np.array_equal(fcm_ref.defuzzify(x, tr.centroids), lab)
    assert np.max(np.abs(tr.centroids - vk)) < 0.05


def test_fixed_point_restart(img1):
    tr = fcm_ref.solve(img1, 4, 2.0, 1e-5, 300)
    again = fcm_ref.solve(img1, 4, 2.0, 1e-5, 300, v0=tr.centroids)
    assert again.T == 1 and again.delta[1] < 1e-5


def test_defuzzify_is_argmax_membership(img1):
    v = np.array([2.8, 41.5, 115.6, 162.2])
    U = fcm_ref.memberships(img1, v, 2.0)
    assert np.array_equal(np.argmax(U, axis=1), fcm_ref.defuzzify(img1, v))
    # ties go to the lowest index
    assert fcm_ref.defuzzify(np.array([50], dtype=np.uint8), np.array([40.0, 60.0])).tolist() == [0]


# --- the brFCM regrouping ---------------------------------------------------------

@pytest.mark.parametrize("m,C", [(2.0, 4), (1.5, 4), (2.5, 4), (2.0, 8), (2.0, 2)])
def test_histogram_regrouping_equals_literal(img1, m, C):
    a = fcm_ref.solve(img1, C, m, 1e-5, 300)
    b = fcm_hist.solve(fcm_hist.histogram(img1), C, m, 1e-5, 300)
    assert a.T == b.T and a.status == b.status
    for t in range(a.T + 1):
        assert _rel(a.v[t], b.v[t]) < 1e-10
        assert abs(a.J[t] - b.J[t]) < 1e-10 * a.J[t]
        if t:
            assert abs(a.delta[t] - b.delta[t]) < 1e-9
    assert np.array_equal(fcm_hist.level_labels(a.centroids)[img1.ravel()],
                          fcm_ref.defuzzify(img1, a.centroids))


def test_constant_image():
    x = np.full(100, 77, dtype=np.uint8)
    tr = fcm_ref.solve(x, 4, 2.0, 1e-5, 300)
    assert tr.T == 1 and tr.status == fcm_ref.OK
    assert tr.centroids.tolist() == [77.0] * 4
    assert tr.delta[1] == 0.0


def test_volume_oracle_converges():
    vol = phantom_3d(16, 32, 32, seed=2)
    tr = fcm_ref.solve(vol, 4, 2.0, 1e-5, 300)
    assert tr.status == fcm_ref.OK and 3 <= tr.T <= 40
