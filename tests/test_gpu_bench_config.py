"""The launch configurations the benchmark times, at full size, against the
oracle: the shipped tuning choices for the 128x128x64 volume (asynchronous
solve that also writes the labels, back to back) and for the 512x512x256
volume, compared iteration by iteration with the level-regrouped FP64 oracle
and the literal one on sampled voxels."""
import os

import numpy as np
import pytest

from oracle import fcm_hist, fcm_ref
from phantom import PhantomParams, phantom
from tests import _parity as P

pytestmark = pytest.mark.gpu

TUNING = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1601_00072_amd",
                      "tuning_mi355x.txt")


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


def shipped(nlog2):
    """driver, grid, unroll, exchange, launch, graph_k of the shipped choice for
    a single C = 4, m = 2 instance of 2^nlog2 .. 2^(nlog2+1) voxels."""
    with open(TUNING) as fh:
        for line in fh:
            f = line.rstrip("\n").split("\t")
            if len(f) == 3 and f[1].startswith("single ") and " C=4 mclass=0 kahan=0 " in f[1] + " " \
                    and f[1].endswith(f"nlog2={nlog2}"):
                v = [int(a) for a in f[2].split()[:6]]
                return dict(driver=v[0], grid=v[1], unroll=v[2], exchange=v[3], launch=v[4], graph_k=v[5])
    pytest.fail(f"no shipped choice for nlog2={nlog2}")


def check(torch, d, x_np, tuning, steps, labels_fused):
    from paper_1601_00072_amd import FCM
    x = torch.from_numpy(x_np.ravel()).to(d)
    lab = torch.empty_like(x)
    with FCM(x, 4) as f:
        f.set_tuning(**tuning)
        got = f.tuning
        assert got["grid"] == tuning["grid"] and got["exchange"] == tuning["exchange"]
        if labels_fused:
            for _ in range(steps):
                f.solve_async(lab)
            res, _ = f.result()
        else:
            res = f.solve()
            f.labels(lab)
        traj = P.gpu_trajectory(f, res.iters)
    h = fcm_hist.histogram(x_np)
    ora = fcm_hist.solve(h, 4, 2.0, 1e-5, 300)
    if res.iters != ora.T:
        ext = fcm_hist.solve(h, 4, 2.0, 0.0, max(res.iters, ora.T) + 1, v0=ora.v[0])
        P.check_iterations(res, ora.T, ext, 1e-5, hist=h, m=2.0, gpu_vs=traj[0])
        ora = ext
    P.compare(res, traj, ora, 1e-5, hist=h, m=2.0)
    lab_np = lab.cpu().numpy()
    P.check_labels(x_np, lab_np, ora.v[res.iters])
    # the literal oracle's memberships and labels on a sample of voxels
    rng = np.random.default_rng(0)
    idx = rng.choice(x_np.size, 20000, replace=False)
    xs = x_np.ravel()[idx]
    assert np.array_equal(fcm_ref.defuzzify(xs, ora.v[res.iters]), lab_np[idx])
    return res


def test_headline_configuration(torch_dev):
    """128x128x64 volume, seed 2: the shipped 2^20 choice, solve and labels in
    one launch, five solves back to back."""
    torch, d = torch_dev
    t = shipped(20)
    announce("bench headline configuration", t)
    x = phantom(PhantomParams(shape=(64, 128, 128), seed=2))
    res = check(torch, d, x, t, 5, True)
    assert res.status == 0 and res.iters == 10


def test_large_volume_configuration(torch_dev):
    """512x512x256 volume, seed 3, sigma 9, bias 20 %: the shipped 2^26 choice."""
    torch, d = torch_dev
    t = shipped(26)
    announce("bench large-volume configuration", t)
    x = phantom(PhantomParams(shape=(256, 512, 512), seed=3, sigma=9.0, bias=0.2))
    res = check(torch, d, x, t, 1, False)
    assert res.status == 0
