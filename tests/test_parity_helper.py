"""CPU checks of the tolerance helper used by the GPU parity tests: the
membership sensitivity it propagates centroid errors with must match finite
differences of the oracle's Eq.4."""
import numpy as np
import pytest

from oracle import fcm_hist
from tests import _parity as P


@pytest.mark.parametrize("m,v", [(2.0, [10.3, 60.7, 61.9, 200.2]), (1.5, [1.9, 36.9, 45.5, 110.7, 120.1, 156.7, 165.7]),
                                 (2.5, [30.0, 90.25, 180.5]), (3.0, [5.5, 250.5])])
def test_sensitivity_matches_finite_differences(m, v):
    v = np.asarray(v)
    levels = np.arange(256)
    h = 1e-6
    best = 0.0
    for x in levels:
        g = np.array([float(x)])
        row = np.zeros(v.size)
        for j in range(v.size):
            vp, vm = v.copy(), v.copy()
            vp[j] += h
            vm[j] -= h
            du = (fcm_hist.level_memberships(g, vp, m) - fcm_hist.level_memberships(g, vm, m)) / (2 * h)
            row += np.abs(du[0])
        best = max(best, float(row.max()))
    got = P.sensitivity(levels, v, m)
    assert got == pytest.approx(best, rel=1e-5)


def test_sensitivity_zero_distance_level_ignored():
    # a grey level sitting exactly on a centroid has u = (1, 0, ...) locally
    # flat in the other centroids and is skipped
    assert P.sensitivity([50], [50.0, 100.0], 2.0) == 0.0


def test_forward_bound_stays_small_where_the_step_contracts():
    """On a well-separated two-level image F contracts from the start: the
    propagated bound stays near step / (1 - rho) and below the 1e-5 bar."""
    x = np.concatenate([np.full(500, 40, np.uint8), np.full(700, 200, np.uint8), np.arange(256, dtype=np.uint8)])
    h = fcm_hist.histogram(x)
    ora = fcm_hist.solve(h, 3, 2.0, 1e-5, 300)
    E = P.forward_bound(h, 2.0, ora, ora.T)
    rel = max(float(np.max(E[t] / np.maximum(np.abs(ora.v[t]), 1.0))) for t in range(ora.T + 1))
    assert 0 < rel < 1e-5


def test_forward_bound_covers_a_perturbed_trajectory():
    """A trajectory perturbed by a relative 2^-24 per step (random signs) stays
    within the propagated bound at every iteration."""
    from phantom import PhantomParams, phantom
    x = phantom(PhantomParams(shape=(96, 96), seed=4011, sigma=8.0)).ravel()
    h = fcm_hist.histogram(x)
    ora = fcm_hist.solve(h, 8, 2.0, 0.0, 80)
    E = P.forward_bound(h, 2.0, ora, 80)
    rng = np.random.default_rng(0)
    v = ora.v[0].copy()
    for t in range(1, 81):
        v = P.level_map(h, v, 2.0) * (1 + 2.0 ** -24 * rng.choice([-1.0, 1.0], size=8))
        assert np.all(np.abs(v - ora.v[t]) <= E[t] + 1e-12), t
