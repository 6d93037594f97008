"""GPU parity of the batched solver: every instance of one persistent launch
against the FP64 oracle at matched iterations, and against the single-instance
path."""
import os

import numpy as np
import pytest

from oracle import fcm_hist
from phantom import PhantomParams, batch_instances, phantom
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


def mixed_instances(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = rng.integers(0, 4)
        if kind == 0:
            shape = (int(rng.integers(1, 9)), int(rng.integers(1, 13)))        # tiny, mostly ragged
        elif kind == 1:
            shape = (int(rng.integers(30, 300)), int(rng.integers(30, 300)))
        elif kind == 2:
            shape = (int(rng.integers(4, 24)), int(rng.integers(16, 64)), int(rng.integers(16, 64)))
        else:
            shape = (int(rng.integers(300, 700)), int(rng.integers(300, 700)))
        C = int(rng.integers(2, 9))
        m = float(rng.choice([2.0, 2.0, 2.0, 1.5, 2.5]))
        params = dict(n_clusters=C, m=m, eps=1e-5, max_iter=300, kahan_only=bool(rng.integers(0, 4) == 0))
        x = phantom(PhantomParams(shape=shape, seed=500 + seed * 1000 + i, sigma=float(rng.uniform(3, 10))))
        out.append((x.ravel(), params))
    return out


def run_batch(torch_dev, items, offset=0, tiling=None):
    torch, dev = torch_dev
    from paper_1601_00072_amd import FCMBatch
    flat = np.concatenate([x for x, _ in items])
    buf = torch.zeros(flat.size + offset + 16, dtype=torch.uint8, device=dev)
    buf[offset:offset + flat.size] = torch.from_numpy(flat).to(dev)
    x = buf[offset:offset + flat.size]
    with FCMBatch(x, [a.size for a, _ in items], [p for _, p in items]) as b:
        if tiling:
            tiling = dict(tiling)
            if "block" in tiling:
                b.set_block(tiling.pop("block"))
            b.set_tiling(**tiling)
        res = b.solve()
        trajs = [[b.trajectory(i, t) for t in range(r.iters + 1)] for i, r in enumerate(res)]
        lab = b.labels().cpu().numpy()
    torch.cuda.synchronize()
    return res, trajs, lab


def check_instance(x, p, res, traj, lab):
    C, m, eps = p["n_clusters"], p.get("m", 2.0), p.get("eps", 1e-5)
    h = fcm_hist.histogram(x)
    if np.count_nonzero(h) <= C:
        # no more grey levels than clusters: clusters collapse onto levels and
        # the zero-distance rule makes the trajectory depend on single-ulp
        # differences (in FP64 too); check the first iteration and validity
        ora = fcm_hist.solve(h, C, m, 0.0, 1)
        for t in range(min(2, res.iters + 1)):
            assert np.max(np.abs(traj[t][0] - ora.v[t]) / np.maximum(np.abs(ora.v[t]), 1.0)) <= P.V_TOL
        assert res.status in (0, 1) and np.all(np.isfinite(res.centroids))
        d = np.abs(x.astype(np.float64)[:, None] - res.centroids[None, :])
        assert np.array_equal(lab, np.argmin(d, axis=1).astype(np.uint8))
        return
    ora = fcm_hist.solve(h, C, m, eps, p.get("max_iter", 300))
    vs = [t[0] for t in traj]
    ds = [t[1] for t in traj]
    Js = [t[2] for t in traj]
    if res.iters != ora.T:
        ext = fcm_hist.solve(h, C, m, 0.0, max(res.iters, ora.T) + 1, v0=ora.v[0])
        P.check_iterations(res, ora.T, ext, eps, hist=h, m=m, gpu_vs=vs)
        ora = ext
    P.compare(res, (vs, ds, Js), ora, eps, hist=h, m=m)
    P.check_labels(x, lab, ora.v[res.iters])
    assert res.passes == res.iters + 1


@pytest.mark.parametrize("seed,offset", [(1, 0), (2, 3), (3, 9)])
def test_batch_mixed_against_oracle(torch_dev, seed, offset):
    items = mixed_instances(24, seed)
    announce("batch mixed seed", seed, "offset", offset, "voxels", sum(x.size for x, _ in items))
    res, trajs, lab = run_batch(torch_dev, items, offset=offset)
    start = 0
    for (x, p), r, tr in zip(items, res, trajs):
        check_instance(x, p, r, tr, lab[start:start + x.size])
        start += x.size


@pytest.mark.parametrize("block,cpt,grid", [(512, 1, 0), (512, 2, 7), (512, 16, 0), (512, 4, 1), (256, 1, 0),
                                            (256, 8, 0), (256, 2, 3), (128, 2, 0), (128, 16, 5)])
def test_batch_tiling(torch_dev, block, cpt, grid):
    items = mixed_instances(12, 7)
    announce("batch tiling block", block, "cpt", cpt, "grid", grid)
    res, trajs, lab = run_batch(torch_dev, items, tiling=dict(block=block, chunks_per_thread=cpt, grid=grid))
    start = 0
    for (x, p), r, tr in zip(items, res, trajs):
        check_instance(x, p, r, tr, lab[start:start + x.size])
        start += x.size


def test_batch_matches_single_instance(torch_dev):
    torch, dev = torch_dev
    from paper_1601_00072_amd import FCM
    items = mixed_instances(10, 11)
    announce("batch vs single")
    res, trajs, lab = run_batch(torch_dev, items)
    for (x, p), r in zip(items, res):
        xt = torch.from_numpy(x).to(dev)
        with FCM(xt, p["n_clusters"], m=p["m"], eps=p["eps"], kahan_only=p["kahan_only"]) as f:
            s = f.solve()
        assert r.status == s.status
        if r.iters == s.iters:
            assert np.max(np.abs(r.centroids - s.centroids) / np.maximum(np.abs(s.centroids), 1.0)) <= 2e-5


def test_batch_repeat_and_determinism(torch_dev):
    torch, dev = torch_dev
    from paper_1601_00072_amd import FCMBatch
    items = mixed_instances(16, 5)
    announce("batch repeat")
    flat = np.concatenate([x for x, _ in items])
    x = torch.from_numpy(flat).to(dev)
    with FCMBatch(x, [a.size for a, _ in items], [p for _, p in items]) as b:
        first = b.solve()
        second = b.solve()
    for a, c in zip(first, second):
        assert a.iters == c.iters and a.status == c.status
        assert np.array_equal(a.centroids, c.centroids)


def shipped_batch_tiling():
    """block, chunks_per_thread and grid of the shipped choice for the batch."""
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1601_00072_amd",
                        "tuning_mi355x.txt")
    with open(path) as fh:
        for line in fh:
            f = line.rstrip("\n").split("\t")
            if len(f) == 3 and f[1].startswith("batch2 ") and " count=512 " in f[1]:
                v = [int(a) for a in f[2].split()[:3]]
                return dict(block=v[0], chunks_per_thread=v[1], grid=v[2])
    pytest.fail("no shipped batch choice")


@pytest.mark.parametrize("which", ["default", "shipped"])
def test_batch_512_instances(torch_dev, which):
    """The batched workload: 496 slices (side U{64..512}) and 16 cubes (side
    U{96..160}), C_i in 3..8, m = 2, all in one launch, with the default
    tiling and with the shipped tuning the benchmark times."""
    inst = batch_instances()
    items = [(phantom(p).ravel(), dict(n_clusters=c, m=2.0, eps=1e-5, max_iter=300)) for p, c in inst]
    tiling = None if which == "default" else shipped_batch_tiling()
    announce("batch 512 instances", sum(x.size for x, _ in items), "voxels, tiling", tiling)
    res, trajs, lab = run_batch(torch_dev, items, tiling=tiling)
    start = 0
    for (x, p), r, tr in zip(items, res, trajs):
        check_instance(x, p, r, tr, lab[start:start + x.size])
        start += x.size


def test_batch_timeline_and_repeat_across_tilings(torch_dev):
    """fcm_batch_timeline: one commit time per phase, increasing; and the
    same tiling gives the same bits in a second launch, after solves under
    another tiling (the instances progress at their own pace, but each
    reduces its rows in tile order)."""
    torch, dev = torch_dev
    from paper_1601_00072_amd import FCMBatch
    items = mixed_instances(20, 13)
    announce("batch timeline")
    flat = np.concatenate([x for x, _ in items])
    x = torch.from_numpy(flat).to(dev)
    with FCMBatch(x, [a.size for a, _ in items], [p for _, p in items]) as b:
        b.set_tiling(chunks_per_thread=1, grid=0)
        first = b.solve()
        for i, r in enumerate(first):
            us = b.timeline(i)
            assert us.shape == (r.passes + 1,)
            assert np.all(np.diff(us) > 0.0) and us[0] >= 0.0
        b.set_tiling(chunks_per_thread=8, grid=0)
        b.solve()
        b.set_block(256)
        b.solve()
        b.set_block(128)
        b.solve()
        b.set_block(512)
        b.set_tiling(chunks_per_thread=1, grid=0)
        again = b.solve()
    for a, c in zip(first, again):
        assert a.iters == c.iters and a.status == c.status and a.J == c.J
        assert np.array_equal(a.centroids, c.centroids)
