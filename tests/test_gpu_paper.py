"""GPU parity of the paper-design baseline (fcm_paper_solve: per-cluster
kernels, Algorithm 2 reductions, host stopping test) against the oracle, for
the paper's random start and the centroid-first starts."""
import numpy as np
import pytest

from oracle import fcm_hist, fcm_ref
from phantom import PhantomParams, phantom, phantom_2d, uniform24
from tests import _parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1601_00072_amd import _lib
    _lib.load()
    return torch, torch.device("cuda:0")


def announce(*what):
    print("CASE", *what, flush=True)


class _Res:
    def __init__(self, iters, status=0):
        self.iters = iters
        self.status = status


def check(torch_dev, x, C, m, eps, init, max_iter=300):
    torch, d = torch_dev
    from paper_1601_00072_amd import paper_baseline
    xt = torch.from_numpy(np.ascontiguousarray(x).ravel()).to(d)
    res, traj, lab, stats = paper_baseline(xt, C, m=m, eps=eps, max_iter=max_iter, init=init, labels=True)
    n = np.asarray(x).size
    random = isinstance(init, tuple)
    if random:
        r = uniform24(init[1], np.arange(n * C, dtype=np.uint64)).reshape(n, C)
        run = lambda e, it: fcm_ref.solve_random_u(x, C, m, e, it, r)
    else:
        v0 = fcm_ref.linspace_init(int(np.min(x)), int(np.max(x)), C) if init is None else \
            np.asarray(init, np.float64).astype(np.float32).astype(np.float64)
        run = lambda e, it: fcm_ref.solve(x, C, m, e, it, v0=v0)
    ora = run(eps, max_iter)
    T_ora = ora.T
    if res.iters != T_ora:
        ora = run(0.0, max(res.iters, T_ora) + 1)
    t0 = 1 if random else 0
    # re-index from t0 so that the helper's bounds start where both sides agree
    sh = fcm_ref.Trajectory(v=ora.v[t0:], delta=[float("nan")] + list(ora.delta[t0 + 1:]), J=ora.J[t0:],
                            T=ora.T - t0, status=ora.status)
    gv = list(traj["v"][t0:])
    hist = fcm_hist.histogram(x)
    if res.iters != T_ora:
        P.check_iterations(_Res(res.iters - t0), T_ora - t0, sh, eps, hist=hist, m=m, gpu_vs=gv)
    bd = P.Bounds(hist, m, sh, gv, res.iters - t0)
    for s in range(res.iters - t0 + 1):
        vo = np.asarray(sh.v[s])
        dv = np.abs(np.asarray(gv[s]) - vo)
        tol = bd.v_tol(s)
        if not np.all(dv <= tol):
            tol = bd.v_tol(s, widen=True)
        assert np.all(dv <= tol), (s + t0, gv[s], vo)
        if s >= 1:
            dd = abs(traj["delta"][s + t0] - sh.delta[s])
            assert dd <= bd.delta_tol(s, sh.delta[s]), (s + t0, traj["delta"][s + t0], sh.delta[s])
    if random:
        # delta^1 against the random U^0
        d1 = abs(traj["delta"][1] - ora.delta[1])
        assert d1 <= P.D_ABS + P.D_REL * ora.delta[1] + bd.sens(0) * bd.err(0), (traj["delta"][1], ora.delta[1])
        assert np.all(np.isnan(traj["v"][0]))
    assert np.isnan(traj["delta"][0]) and np.isnan(res.J)
    P.check_labels(x, lab, ora.v[res.iters])
    assert stats["launches"] == 5 * C * res.iters
    assert stats["kernels_ms"] > 0 and stats["copy_ms"] > 0 and stats["total_ms"] >= stats["host_ms"]
    return res, stats


@pytest.mark.parametrize("C,m", [(4, 2.0), (3, 2.5), (6, 1.5)])
def test_random_start_paper_eps(torch_dev, C, m):
    announce("paper design random start C", C, "m", m)
    x = phantom_2d(200, 200, seed=1)
    check(torch_dev, x, C, m, 0.005, ("random_u", 40 + C))


@pytest.mark.parametrize("C,m", [(4, 2.0), (2, 2.0), (5, 1.5), (8, 2.5)])
def test_linspace_start(torch_dev, C, m):
    announce("paper design linspace C", C, "m", m)
    x = phantom_2d(160, 250, seed=7)   # 40,000 pixels: 157 partial sums, ragged last block
    check(torch_dev, x, C, m, 1e-5, None)


def test_given_start_ragged_volume(torch_dev):
    announce("paper design given start, ragged volume")
    x = phantom(PhantomParams(shape=(13, 97, 61), seed=5)).ravel()[:76_913]
    check(torch_dev, x, 4, 2.0, 1e-4, [10.5, 60.0, 100.25, 170.0])


@pytest.mark.parametrize("n", [1, 255, 256, 257, 513])
def test_small_sizes(torch_dev, n):
    announce("paper design n", n)
    rng = np.random.default_rng(n)
    x = rng.integers(0, 256, n).astype(np.uint8)
    if n == 1:
        torch, d = torch_dev
        from paper_1601_00072_amd import paper_baseline
        res, traj, lab, _ = paper_baseline(torch.from_numpy(x).to(d), 3, init=None, labels=True)
        assert res.status == 0 and lab[0] == 0
        return
    check(torch_dev, x, 3, 2.0, 1e-4, None)


def test_max_iter(torch_dev):
    announce("paper design max_iter")
    x = phantom_2d(96, 96, seed=9)
    res, _ = check(torch_dev, x, 6, 2.0, 1e-9, None, max_iter=2)
    assert res.iters == 2 and res.status == 1
