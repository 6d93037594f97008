"""The learned warm start at its full workload size: the network trained on
the GPU-converged centroids of 20,000 jittered 256x256 phantoms, evaluated on
1,024 held-out 256x256 phantoms and 64 held-out 128^3 volumes, one handle per
instance and all in one batched launch.

Asserted: training converges; on both held-out sets the warm start takes
fewer iterations on average; every accepted warm result reaches the plain
J_m within 1e-6 relative; where the warm result is refused, the batch returns
the plain result itself.  Wall times are printed, not asserted.
"""
import multiprocessing as mp
from multiprocessing import shared_memory

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

J_REL = 1e-6


def _fill(job):
    """Worker (spawned: it touches no GPU): phantoms of one shape into the
    shared block at the given byte offsets."""
    name, shape, seeds, offs = job
    from phantom import jittered_params, phantom
    shm = shared_memory.SharedMemory(name=name)
    try:
        view = np.ndarray((shm.size,), dtype=np.uint8, buffer=shm.buf)
        n = int(np.prod(shape))
        for sd, o in zip(seeds, offs):
            view[o:o + n] = phantom(jittered_params(shape, sd)).ravel()
        del view
    finally:
        shm.close()
    return len(seeds)


def generate(shape, count, seed0, workers=16):
    """count phantoms of `shape` (seeds seed0 + i) as one flat uint8 array,
    built by spawned worker processes."""
    n = int(np.prod(shape))
    shm = shared_memory.SharedMemory(create=True, size=n * count)
    try:
        step = max(1, min(250, count // workers))
        jobs = [(shm.name, shape, [seed0 + i for i in range(i0, min(count, i0 + step))],
                 [i * n for i in range(i0, min(count, i0 + step))]) for i0 in range(0, count, step)]
        with mp.get_context("spawn").Pool(min(workers, len(jobs))) as pool:
            assert sum(pool.map(_fill, jobs, chunksize=1)) == count
        out = np.ndarray((n * count,), dtype=np.uint8, buffer=shm.buf).copy()
    finally:
        shm.close()
        shm.unlink()
    return out


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1601_00072_amd import _lib
    _lib.load()
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def trained(torch_dev):
    torch, d = torch_dev
    from paper_1601_00072_amd import learn
    print("CASE learned start, 20,000 training phantoms 256x256", flush=True)
    train = generate((256, 256), 20000, 10 ** 6)
    x = torch.from_numpy(train).to(d)
    net, losses, t_tgt, t_train = learn.train(x, [256 * 256] * 20000, C=4, epochs=100, batch=256, lr=1e-3, seed=1)
    print(f"training loss {losses[0]:.3e} -> {losses[-1]:.3e}; targets {t_tgt:.2f} s, training {t_train:.2f} s",
          flush=True)
    del x
    yield net, losses
    net.close()


def check_batch_rule(torch, d, net, flat, sizes):
    """One batched launch with the fall-back check: accepted warm results
    within the J_m rule, refused ones equal to the plain result."""
    from paper_1601_00072_amd import FCMBatch
    params = [dict(n_clusters=4, m=2.0, eps=1e-5)] * len(sizes)
    with FCMBatch(torch.from_numpy(flat).to(d), sizes, params) as b:
        warm, used, plain = b.solve_warm(net, check=True)
    iw = np.array([r.iters for r, u, p in zip(warm, used, plain)])
    ip = np.array([p.iters for p in plain])
    for r, u, p in zip(warm, used, plain):
        assert r.status == 0 and p.status == 0
        if u:
            assert r.J <= p.J * (1.0 + J_REL)
        else:
            assert r.iters == p.iters and np.array_equal(r.centroids, p.centroids)
    return iw, ip, used


@pytest.mark.parametrize("name,shape,count,seed0", [("slices", (256, 256), 1024, 2 * 10 ** 6),
                                                    ("volumes", (128, 128, 128), 64, 3 * 10 ** 6)])
def test_learned_start_full_size(torch_dev, trained, name, shape, count, seed0):
    torch, d = torch_dev
    from paper_1601_00072_amd import learn
    net, losses = trained
    assert losses[-1] < 0.01 * losses[0]
    print("CASE learned start held-out", name, count, flush=True)
    flat = generate(shape, count, seed0)
    sizes = [int(np.prod(shape))] * count
    ev = learn.evaluate_instances(net, torch.from_numpy(flat).to(d), sizes, C=4)
    print(name, "one handle each:", ev, flush=True)
    assert ev["iters_warm_mean"] < ev["iters_plain_mean"]
    assert ev["max_rel_J_excess_accepted"] <= J_REL
    assert ev["fallback_rate"] <= 0.05
    iw, ip, used = check_batch_rule(torch, d, net, flat, sizes)
    eff = np.where(used, iw, ip)
    print(name, "batched: mean iterations plain", ip.mean(), "warm", eff.mean(), "fall-backs", int((~used).sum()),
          flush=True)
    assert eff.mean() < ip.mean()
