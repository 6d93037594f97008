"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by element.

Every case prints its name, shape and parameters before touching the GPU.
"""
import numpy as np
import pytest

from oracle import fcm_hist, fcm_ref
from phantom import PhantomParams, phantom, phantom_2d, phantom_3d
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


def run_gpu(torch_dev, x_np, C, m=2.0, eps=1e-5, max_iter=300, init=None, offset=0, **kw):
    torch, dev = torch_dev
    from paper_1601_00072_amd import FCM
    flat = np.ascontiguousarray(x_np).ravel()
    buf = torch.zeros(flat.size + offset + 16, dtype=torch.uint8, device=dev)
    buf[offset:offset + flat.size] = torch.from_numpy(flat).to(dev)
    x = buf[offset:offset + flat.size]
    tuning = kw.pop("tuning", None)
    f = FCM(x, C, m=m, eps=eps, max_iter=max_iter, init=init, **kw)
    if tuning:
        f.set_tuning(**tuning)
    res = f.solve()
    traj = P.gpu_trajectory(f, res.iters)
    lab = f.labels().cpu().numpy()
    torch.cuda.synchronize()
    f.close()
    return res, traj, lab


def check_against_literal(torch_dev, x, C, m=2.0, eps=1e-5, max_iter=300, init=None, **kw):
    res, traj, lab = run_gpu(torch_dev, x, C, m, eps, max_iter, init, **kw)
    v0 = None if init is None else np.asarray(init, dtype=np.float64).astype(np.float32).astype(np.float64)
    ora = fcm_ref.solve(x, C, m, eps, max_iter, v0=v0)
    assert res.status in (0, 1)
    if res.iters != ora.T:
        ora_ext = fcm_ref.solve(x, C, m, 0.0, max(res.iters, ora.T) + 1, v0=ora.v[0])
        P.check_iterations(res, ora.T, ora_ext, eps, hist=fcm_hist.histogram(x), m=m, gpu_vs=traj[0])
        ora = ora_ext
    err = P.compare(res, traj, ora, eps, hist=fcm_hist.histogram(x), m=m)
    amb = P.check_labels(x, lab, ora.v[res.iters])
    assert res.passes == res.iters + 1
    return res, ora, err, amb


# --- the two small workloads ---------------------------------------------------

def test_slice_200x200_c4_m2(torch_dev):
    announce("slice 200x200 seed 1, C=4 m=2")
    x = phantom_2d(200, 200, seed=1)
    res, ora, err, amb = check_against_literal(torch_dev, x, 4)
    assert res.status == 0 and res.iters == ora.T
    assert amb == 0
    print("errors", err, "ambiguous levels", amb, "T", res.iters)


def test_volume_64x128x128_c4_m2(torch_dev):
    announce("volume 64x128x128 seed 2, C=4 m=2")
    x = phantom_3d(64, 128, 128, seed=2)
    res, ora, err, amb = check_against_literal(torch_dev, x, 4)
    assert res.status == 0
    assert amb == 0
    print("errors", err, "ambiguous levels", amb, "T", res.iters)


def test_volume_kahan_only(torch_dev):
    announce("volume 64x128x128 seed 2, C=4 m=2, compensated FP32 cross-block")
    x = phantom_3d(64, 128, 128, seed=2)
    check_against_literal(torch_dev, x, 4, kahan_only=True)


# --- sizes, alignment and tails -----------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 33, 255, 4096, 4097, 65537, 262147])
@pytest.mark.parametrize("offset", [0, 1, 7])
def test_ragged_sizes_and_offsets(torch_dev, n, offset):
    announce("ragged n", n, "offset", offset)
    x = phantom_2d(520, 520, seed=9).ravel()[:n].copy()
    check_against_literal(torch_dev, x, 4)


@pytest.mark.parametrize("driver,exchange", [(0, 0), (2, 1), (2, 2), (2, 3)])
@pytest.mark.parametrize("grid,unroll", [(1, 1), (3, 2), (77, 1), (256, 2), (1024, 1), (4096, 2)])
def test_launch_shapes(torch_dev, grid, unroll, driver, exchange):
    announce("launch grid", grid, "unroll", unroll, "driver", driver, "exchange", exchange)
    x = phantom_2d(300, 333, seed=4)
    check_against_literal(torch_dev, x, 4, tuning=dict(grid=grid, unroll=unroll, driver=driver, exchange=exchange))


@pytest.mark.parametrize("driver,k,exchange,launch", [(0, 1, 0, 0), (0, 5, 0, 0), (1, 1, 0, 0), (1, 3, 0, 0),
                                                      (1, 16, 0, 0), (2, 1, 0, 0), (2, 1, 1, 0), (2, 1, 2, 0),
                                                      (2, 1, 0, 1), (2, 1, 1, 1), (2, 1, 2, 1), (2, 1, 3, 0),
                                                      (2, 1, 3, 1), (2, 3, 3, 1)])
@pytest.mark.parametrize("shape", [(200, 200), (32, 160, 160)])
def test_drivers(torch_dev, driver, k, exchange, launch, shape):
    announce("driver", driver, "graph_k", k, "exchange", exchange, "launch", launch, "shape", shape)
    x = phantom(PhantomParams(shape=shape, seed=1))
    check_against_literal(torch_dev, x, 4, tuning=dict(driver=driver, graph_k=k, exchange=exchange, launch=launch))


@pytest.mark.parametrize("C,m", [(2, 2.0), (5, 1.5), (8, 2.5), (7, 3.0)])
def test_two_level_exchange_clusters(torch_dev, C, m):
    """The exchange through the XCDs across cluster counts and fuzziness (FP64
    sums in another fixed order than the one-level exchanges)."""
    announce("two-level exchange C", C, "m", m)
    x = phantom(PhantomParams(shape=(48, 128, 128), seed=10 + C))
    check_against_literal(torch_dev, x, C, m=m, tuning=dict(driver=2, exchange=3))


def test_two_level_exchange_after_odd_dispatches(torch_dev):
    """Launches of 1..9 blocks in between move the XCD the next launch starts
    on; the two-level solves (or their fallback) still match the oracle."""
    torch, dev = torch_dev
    from paper_1601_00072_amd import FCM
    announce("two-level exchange after odd dispatches")
    x = phantom_2d(200, 200, seed=1)
    ref = fcm_ref.solve(x, 4, 2.0, 1e-5, 300)
    xt = torch.from_numpy(x.ravel()).to(dev)
    for blocks in range(1, 10):
        y = torch.from_numpy(np.arange(blocks * 4096, dtype=np.int64) % 251).to(dev).to(torch.uint8)
        with FCM(y, 3) as g:
            g.set_tuning(driver=2, grid=blocks, exchange=1)
            g.solve()
        with FCM(xt, 4) as f:
            f.set_tuning(driver=2, exchange=3)
            r = f.solve()
        assert r.iters == ref.T
        assert np.max(np.abs(r.centroids - ref.v[ref.T]) / np.maximum(np.abs(ref.v[ref.T]), 1.0)) <= 1e-5


# --- cluster counts and fuzziness -------------------------------------------

@pytest.mark.parametrize("C", [2, 3, 4, 5, 6, 7, 8])
def test_cluster_counts_m2(torch_dev, C):
    announce("slice 128x160 seed 12, m=2, C", C)
    x = phantom_2d(128, 160, seed=12)
    check_against_literal(torch_dev, x, C)


@pytest.mark.parametrize("m", [1.5, 2.5, 3.0, 1.25])
@pytest.mark.parametrize("C", [3, 4, 8])
def test_fuzziness(torch_dev, m, C):
    announce("slice 128x128 seed 13, m", m, "C", C)
    x = phantom_2d(128, 128, seed=13)
    check_against_literal(torch_dev, x, C, m=m)


# --- degenerate cases -----------------------------------------------------------

def test_constant_image(torch_dev):
    announce("constant image")
    x = np.full(5000, 77, dtype=np.uint8)
    res, traj, lab = run_gpu(torch_dev, x, 4)
    assert res.status == 0 and res.iters == 1
    assert res.centroids.tolist() == [77.0] * 4
    assert traj[1][1] == 0.0
    assert np.all(lab == 0)


def test_two_levels_exact(torch_dev):
    announce("two levels")
    x = np.array([30] * 500 + [170] * 700, dtype=np.uint8)
    res, traj, lab = run_gpu(torch_dev, x, 2)
    assert res.status == 0 and res.iters == 1
    assert res.centroids.tolist() == [30.0, 170.0]
    assert np.array_equal(lab, (x == 170).astype(np.uint8))


def test_fewer_voxels_than_clusters(torch_dev):
    """n < C: clusters without support collapse onto data levels, so after the
    first update several centroids coincide and the zero-distance rule makes the
    trajectory depend on single-ulp differences (in FP64 too).  Element parity
    is checked for the first iteration; after that the result must be valid and
    self-consistent."""
    announce("n=3 < C=8")
    x = np.array([10, 200, 90], dtype=np.uint8)
    res, traj, lab = run_gpu(torch_dev, x, 8)
    ora = fcm_ref.solve(x, 8, 2.0, 0.0, 1)
    for t in range(min(2, res.iters + 1)):
        assert np.max(np.abs(traj[0][t] - ora.v[t]) / np.maximum(np.abs(ora.v[t]), 1.0)) <= P.V_TOL
    assert res.status in (0, 1)
    assert np.all(np.isfinite(res.centroids))
    assert np.all(res.centroids >= 10.0 - 1e-3) and np.all(res.centroids <= 200.0 + 1e-3)
    d = np.abs(x.astype(np.float64)[:, None] - res.centroids[None, :])
    assert np.array_equal(lab, np.argmin(d, axis=1).astype(np.uint8))


def test_voxel_on_centroid_gets_full_membership(torch_dev):
    """linspace puts v_0 on the minimum level; the pass must treat the zero
    distance as membership 1 (otherwise v^1 would differ)."""
    announce("zero distance")
    x = np.array([0] * 100 + [50] * 10 + [255] * 100, dtype=np.uint8)
    check_against_literal(torch_dev, x, 3)


def test_max_iter_not_converged(torch_dev):
    announce("max_iter 3")
    x = phantom_2d(200, 200, seed=1)
    res, ora, err, amb = check_against_literal(torch_dev, x, 4, max_iter=3)
    assert res.status == 1 and res.iters == 3


def test_given_init(torch_dev):
    announce("given init")
    x = phantom_2d(200, 200, seed=1)
    check_against_literal(torch_dev, x, 4, init=[10.3, 60.1, 100.7, 180.25])


# --- behaviour of the handle ------------------------------------------------------

def test_bitwise_deterministic(torch_dev):
    announce("determinism")
    x = phantom_3d(32, 96, 96, seed=21)
    a = run_gpu(torch_dev, x, 5)
    b = run_gpu(torch_dev, x, 5)
    assert a[0].iters == b[0].iters
    for t in range(a[0].iters + 1):
        assert np.array_equal(a[1][0][t], b[1][0][t])
        assert a[1][2][t] == b[1][2][t]
    assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("driver", [0, 1, 2])
def test_iterate_in_steps_equals_solve(torch_dev, driver):
    announce("iterate steps, driver", driver)
    torch, dev = torch_dev
    from paper_1601_00072_amd import FCM
    x = torch.from_numpy(phantom_2d(200, 200, seed=1).ravel()).to(dev)
    with FCM(x, 4) as f:
        f.set_tuning(driver=driver)
        full = f.solve()
    with FCM(x, 4) as f:
        f.set_tuning(driver=driver)
        seen = []
        while True:
            r = f.iterate(1)
            seen.append(r.passes)
            if r.status != 2:
                break
        assert r.iters == full.iters and np.array_equal(r.centroids, full.centroids)
        assert seen == list(range(1, full.passes + 1))


def test_labels_to_misaligned_buffer(torch_dev):
    announce("labels to misaligned buffer")
    torch, dev = torch_dev
    from paper_1601_00072_amd import FCM
    xn = phantom_2d(123, 457, seed=3).ravel()
    x = torch.from_numpy(xn).to(dev)
    out = torch.zeros(xn.size + 3, dtype=torch.uint8, device=dev)
    with FCM(x, 4) as f:
        res = f.solve()
        f.labels(out[3:])
        a = out[3:].cpu().numpy()
        b = f.labels().cpu().numpy()
    assert np.array_equal(a, b)
    P.check_labels(xn, a, res.centroids)


def test_timing_flag(torch_dev):
    announce("timing")
    torch, dev = torch_dev
    from paper_1601_00072_amd import FCM
    x = torch.from_numpy(phantom_3d(64, 128, 128, seed=2).ravel()).to(dev)
    with FCM(x, 4, timing=True) as f:
        r = f.solve()
    assert r.kernel_ms > 0.0 and r.passes == r.iters + 1


# --- full-size large volumes: level-regrouped oracle --------------------------------

def check_against_levels(torch_dev, x, C, m, eps=1e-5, **kw):
    res, traj, lab = run_gpu(torch_dev, x, C, m, eps, **kw)
    h = fcm_hist.histogram(x)
    ora = fcm_hist.solve(h, C, m, eps, 300)
    if res.iters != ora.T:
        ora_ext = fcm_hist.solve(h, C, m, 0.0, max(res.iters, ora.T) + 1, v0=ora.v[0])
        P.check_iterations(res, ora.T, ora_ext, eps, hist=h, m=m, gpu_vs=traj[0])
        ora = ora_ext
    err = P.compare(res, traj, ora, eps, hist=h, m=m)
    amb = P.check_labels(x, lab, ora.v[res.iters])
    return res, err, amb


@pytest.mark.parametrize("sigma,C,m,kahan", [(9.0, 4, 2.0, False), (3.0, 8, 2.5, False), (9.0, 8, 1.5, True),
                                             (3.0, 4, 2.0, True)])
def test_volume_181x217x181(torch_dev, sigma, C, m, kahan):
    announce("volume 181x217x181 sigma", sigma, "C", C, "m", m, "kahan_only", kahan)
    x = phantom(PhantomParams(shape=(181, 217, 181), seed=3, sigma=sigma, bias=0.2))
    res, err, amb = check_against_levels(torch_dev, x, C, m, kahan_only=kahan)
    assert amb == 0
    print("T", res.iters, "errors", err, "ambiguous", amb)


def test_volume_512x512x256(torch_dev):
    announce("volume 512x512x256 sigma 9, C=4 m=2")
    x = phantom(PhantomParams(shape=(256, 512, 512), seed=3, sigma=9.0, bias=0.2))
    res, err, amb = check_against_levels(torch_dev, x, 4, 2.0)
    assert amb == 0
    print("T", res.iters, "errors", err, "ambiguous", amb)
