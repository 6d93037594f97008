"""GPU parity of the histogram-domain driver (FCM_DRIVER_HISTOGRAM): one
histogram pass, then Algorithm 1 over the grey levels in FP64 -- compared
with the FP64 level-regrouped oracle (and the literal oracle on small
inputs) at FP64 tolerances, iteration by iteration."""
import numpy as np
import pytest

from oracle import fcm_hist, fcm_ref
from phantom import PhantomParams, phantom, phantom_2d

pytestmark = pytest.mark.gpu

# FP64 on both sides; only the summation order differs (256 levels)
V_REL, J_REL, D_ABS = 1e-10, 1e-11, 1e-11


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


def run_levels(torch_dev, x, C, m=2.0, eps=1e-5, max_iter=300, init=None, offset=0, steps=None):
    torch, d = torch_dev
    from paper_1601_00072_amd import FCM
    flat = np.ascontiguousarray(x).ravel()
    buf = torch.zeros(flat.size + offset + 16, dtype=torch.uint8, device=d)
    buf[offset:offset + flat.size] = torch.from_numpy(flat).to(d)
    xt = buf[offset:offset + flat.size]
    with FCM(xt, C, m=m, eps=eps, max_iter=max_iter, init=init) as f:
        f.set_tuning(driver=3)
        if steps:
            r = None
            for _ in range(max_iter + 2):
                r = f.iterate(steps)
                if r.status != 2:
                    break
        else:
            r = f.solve()
        traj = [f.trajectory(t) for t in range(r.iters + 1)]
        lab = f.labels().cpu().numpy()
    return r, traj, lab


def check(x, C, r, traj, lab, m=2.0, eps=1e-5, max_iter=300, init=None):
    h = fcm_hist.histogram(x)
    v0 = None if init is None else np.asarray(init, np.float64).astype(np.float32).astype(np.float64)
    ora = fcm_hist.solve(h, C, m, eps, max_iter, v0=v0)
    if r.iters != ora.T:
        # FP64 on both sides: a different stopping point needs delta within
        # rounding of eps
        ext = fcm_hist.solve(h, C, m, 0.0, max(r.iters, ora.T) + 1, v0=ora.v[0])
        for t in range(min(r.iters, ora.T), max(r.iters, ora.T)):
            assert abs(ext.delta[t] - eps) <= 1e-9, (r.iters, ora.T, ext.delta[t])
        ora = ext
    for t in range(r.iters + 1):
        v, dlt, J = traj[t]
        vo = ora.v[t]
        assert np.max(np.abs(v - vo) / np.maximum(np.abs(vo), 1.0)) <= V_REL, (t, v, vo)
        assert abs(J - ora.J[t]) <= J_REL * ora.J[t] + 1e-9, (t, J, ora.J[t])
        if t > 0:
            assert abs(dlt - ora.delta[t]) <= D_ABS, (t, dlt, ora.delta[t])
    assert np.array_equal(lab, fcm_hist.level_labels(ora.v[r.iters])[np.asarray(x).ravel()])
    assert r.passes == r.iters + 1
    return ora


def test_slice_against_literal_oracle(torch_dev):
    announce("levels slice 200x200 vs literal")
    x = phantom_2d(200, 200, seed=1)
    r, traj, lab = run_levels(torch_dev, x, 4)
    lit = fcm_ref.solve(x, 4, 2.0, 1e-5, 300)
    assert r.status == 0 and r.iters == lit.T
    assert np.max(np.abs(r.centroids - lit.v[lit.T]) / np.abs(lit.v[lit.T])) <= 1e-10
    check(x, 4, r, traj, lab)


@pytest.mark.parametrize("C", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("m", [2.0, 1.5, 2.5, 3.0])
def test_clusters_and_fuzziness(torch_dev, C, m):
    announce("levels C", C, "m", m)
    x = phantom(PhantomParams(shape=(40, 96, 96), seed=5 + C))
    r, traj, lab = run_levels(torch_dev, x, C, m=m)
    check(x, C, r, traj, lab, m=m)


@pytest.mark.parametrize("offset", [0, 1, 7])
def test_volume_unaligned(torch_dev, offset):
    announce("levels volume offset", offset)
    x = phantom(PhantomParams(shape=(64, 128, 128), seed=2))
    r, traj, lab = run_levels(torch_dev, x, 4, offset=offset)
    check(x, 4, r, traj, lab)


def test_large_volume(torch_dev):
    announce("levels 512x512x256")
    x = phantom(PhantomParams(shape=(256, 512, 512), seed=3, sigma=9.0, bias=0.2))
    r, traj, lab = run_levels(torch_dev, x, 8, m=2.5)
    check(x, 8, r, traj, lab, m=2.5)


@pytest.mark.parametrize("case", ["constant", "two_levels", "tiny", "max_iter", "given", "steps"])
def test_special_cases(torch_dev, case):
    announce("levels", case)
    rng = np.random.default_rng(3)
    kw = {}
    if case == "constant":
        x = np.full((50, 60), 77, np.uint8)
        C = 3
    elif case == "two_levels":
        x = np.where(rng.random((64, 64)) < 0.3, 20, 200).astype(np.uint8)
        C = 2
    elif case == "tiny":
        x = np.array([5, 9, 200], np.uint8)
        C = 4
    elif case == "max_iter":
        x = phantom_2d(96, 96, seed=9)
        C, kw = 6, dict(max_iter=3)
    elif case == "given":
        x = phantom_2d(128, 128, seed=4)
        C, kw = 4, dict(init=[3.3, 50.0, 99.5, 180.25])
    else:
        x = phantom_2d(128, 96, seed=6)
        C, kw = 4, dict(steps=3)
    r, traj, lab = run_levels(torch_dev, x, C, **kw)
    kw.pop("steps", None)
    if case == "tiny":
        # fewer grey levels than clusters: the zero-distance rule makes the
        # trajectory sensitive to single-ulp differences; first step + validity
        h = fcm_hist.histogram(x)
        ora = fcm_hist.solve(h, C, 2.0, 0.0, 1)
        assert np.allclose(traj[0][0], ora.v[0]) and np.allclose(traj[min(1, r.iters)][0], ora.v[min(1, r.iters)])
        assert r.status in (0, 1) and np.all(np.isfinite(r.centroids))
        return
    check(x, C, r, traj, lab, **kw)
    if case == "max_iter":
        assert r.iters == 3 and r.status == 1
