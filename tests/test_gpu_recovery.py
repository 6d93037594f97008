"""The failure path of the persistent driver's cross-block waits, driven from
the host: a wait limit far below a pass's duration makes every wait give up
(each kernel still ends normally: a wait that expires sets the shared abort
word, which every other wait watches).  A resident solve that gives up is
solved again from its start in a cooperative launch; a cooperative or
asynchronous solve that gives up reports FCM_EDEVICE; either way the handle
recovers and the next solve matches the oracle."""
import numpy as np
import pytest

from oracle import fcm_hist
from phantom import PhantomParams, phantom
from tests import _parity as P

pytestmark = pytest.mark.gpu

TINY = 1e-8      # about one tick of the 100 MHz wall clock: every wait gives up
DEFAULT = 5.0


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1601_00072_amd import _lib
    _lib.load()
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def volume(torch_dev):
    torch, d = torch_dev
    x = phantom(PhantomParams(shape=(64, 128, 128), seed=2))
    h = fcm_hist.histogram(x)
    ora = fcm_hist.solve(h, 4, 2.0, 1e-5, 300)
    return x.ravel(), torch.from_numpy(x.ravel()).to(d), h, ora


def check(f, res, x_np, h, ora, lab):
    assert res.status == 0
    traj = P.gpu_trajectory(f, res.iters)
    if res.iters != ora.T:
        ext = fcm_hist.solve(h, 4, 2.0, 0.0, max(res.iters, ora.T) + 1, v0=ora.v[0])
        P.check_iterations(res, ora.T, ext, 1e-5, hist=h, m=2.0, gpu_vs=traj[0])
        ora = ext
    P.compare(res, traj, ora, 1e-5, hist=h, m=2.0)
    P.check_labels(x_np, lab, ora.v[res.iters])


def test_resident_solve_that_gives_up_is_solved_again_cooperatively(torch_dev, volume):
    from paper_1601_00072_amd import FCM
    x_np, x, h, ora = volume
    print("CASE resident launch, wait limit", TINY, flush=True)
    with FCM(x, 4) as f:
        f.set_tuning(driver=2, launch=1, grid=256)
        assert f.set_wait_limit(TINY) == 0
        res = f.solve()                   # first launch gives up, the cooperative one finishes
        assert f.set_wait_limit(0) == 1
        check(f, res, x_np, h, ora, f.labels().cpu().numpy())
        f.set_wait_limit(DEFAULT)
        f.reset()
        res2 = f.solve()                  # the handle goes on with resident launches
        assert f.set_wait_limit(0) == 1
        assert res2.iters == res.iters and np.array_equal(res2.centroids, res.centroids)


def test_cooperative_solve_that_gives_up_reports_and_recovers(torch_dev, volume):
    from paper_1601_00072_amd import FCM
    from paper_1601_00072_amd.api import FcmError
    x_np, x, h, ora = volume
    print("CASE cooperative launch, wait limit", TINY, flush=True)
    with FCM(x, 4) as f:
        f.set_tuning(driver=2, launch=0, grid=256)
        f.set_wait_limit(TINY)
        with pytest.raises(FcmError) as e:
            f.solve()
        assert e.value.status == -3
        assert f.set_wait_limit(DEFAULT) == 0
        f.reset()
        res = f.solve()
        check(f, res, x_np, h, ora, f.labels().cpu().numpy())


def test_async_solve_that_gives_up_reports_and_recovers(torch_dev, volume):
    torch, d = torch_dev
    from paper_1601_00072_amd import FCM
    from paper_1601_00072_amd.api import FcmError
    x_np, x, h, ora = volume
    print("CASE asynchronous solve, wait limit", TINY, flush=True)
    lab = torch.empty_like(x)
    with FCM(x, 4) as f:
        f.set_tuning(driver=2, launch=1, grid=256)
        f.set_wait_limit(TINY)
        f.solve_async(lab)
        with pytest.raises(FcmError) as e:
            f.result()
        assert e.value.status == -3
        f.set_wait_limit(DEFAULT)
        f.solve_async(lab)
        f.solve_async(lab)
        res, _ = f.result()
        check(f, res, x_np, h, ora, lab.cpu().numpy())


def test_wait_limit_validation(torch_dev, volume):
    from paper_1601_00072_amd import FCM
    from paper_1601_00072_amd.api import FcmError
    _, x, _, _ = volume
    with FCM(x, 4) as f:
        for bad in (-1.0, 61.0, float("nan"), float("inf")):
            with pytest.raises(FcmError):
                f.set_wait_limit(bad)
