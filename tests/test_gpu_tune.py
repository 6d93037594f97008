"""GPU tests of the autotuner: the configuration it picks still matches the
FP64 oracle, and its cache file is written once and reused."""
import numpy as np
import pytest

from oracle import fcm_hist
from phantom import PhantomParams, phantom
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


def check_levels(f, x, C, m=2.0, eps=1e-5):
    res = f.solve()
    traj = P.gpu_trajectory(f, res.iters)
    h = fcm_hist.histogram(x)
    ora = fcm_hist.solve(h, C, m, eps, 300)
    if res.iters != ora.T:
        ext = fcm_hist.solve(h, C, m, 0.0, max(res.iters, ora.T) + 1, v0=ora.v[0])
        P.check_iterations(res, ora.T, ext, eps, hist=h, m=m, gpu_vs=traj[0])
        ora = ext
    P.compare(res, traj, ora, eps, hist=h, m=m)
    P.check_labels(x, f.labels().cpu().numpy(), ora.v[res.iters])
    return res


@pytest.mark.parametrize("shape,C", [((64, 128, 128), 4), ((200, 200), 4), ((40, 181, 217), 8)])
def test_autotune_keeps_parity_and_caches(torch_dev, tmp_path, shape, C):
    torch, d = torch_dev
    from paper_1601_00072_amd import FCM
    announce("autotune", shape, C)
    x = phantom(PhantomParams(shape=shape, seed=2)).ravel()
    xt = torch.from_numpy(x).to(d)
    cache = tmp_path / "tune.txt"
    with FCM(xt, C) as f:
        tun, ms = f.autotune(cache=cache, reps=2)
        print("chosen", tun, f"{ms:.3f} ms")
        assert ms > 0 and f.tuning == tun
        check_levels(f, x, C)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("fcm-tune1\tsingle ")
    # a second handle of the same class takes the cached choice without timing
    with FCM(xt, C) as g:
        tun2, ms2 = g.autotune(cache=cache, reps=2)
        assert tun2 == tun and ms2 == pytest.approx(ms)
        check_levels(g, x, C)
    assert len(cache.read_text().splitlines()) == 1


def test_batch_autotune_keeps_parity(torch_dev, tmp_path):
    torch, d = torch_dev
    from paper_1601_00072_amd import FCMBatch
    from tests.test_gpu_batch import check_instance, mixed_instances
    announce("batch autotune")
    items = mixed_instances(16, 21)
    flat = torch.from_numpy(np.concatenate([x for x, _ in items])).to(d)
    cache = tmp_path / "tune.txt"
    with FCMBatch(flat, [x.size for x, _ in items], [p for _, p in items]) as b:
        bs, cpt, grid, ms = b.autotune(cache=cache, reps=2)
        print("chosen block and tiling", bs, cpt, grid, f"{ms:.3f} ms")
        assert bs in (128, 256, 512) and cpt in (1, 2, 3, 4, 5, 6, 8, 12, 16) and ms > 0
        res = b.solve()
        trajs = [[b.trajectory(i, t) for t in range(r.iters + 1)] for i, r in enumerate(res)]
        lab = b.labels().cpu().numpy()
    start = 0
    for (x, p), r, tr in zip(items, res, trajs):
        check_instance(x, p, r, tr, lab[start:start + x.size])
        start += x.size
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("fcm-tune1\tbatch2 ")
