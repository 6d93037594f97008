"""GPU parity of the segmentation-quality kernels (Sec. 5.2.2, Eq.5):
confusion counts bit-exact against the oracle, Dice coefficients bit-exact
(one rounding of the same exact integers on both sides), and the Dice
scores of GPU segmentations of phantoms against the oracle's."""
import numpy as np
import pytest

from oracle import dice as odice
from oracle import fcm_ref
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


def on_device(torch, d, a, offset):
    """a (uint8) placed at byte offset `offset` of a fresh device buffer."""
    buf = torch.zeros(a.size + offset + 32, dtype=torch.uint8, device=d)
    buf[offset:offset + a.size] = torch.from_numpy(np.ascontiguousarray(a).ravel()).to(d)
    return buf[offset:offset + a.size]


@pytest.mark.parametrize("n", [1, 15, 16, 17, 4099, (1 << 20) + 13])
@pytest.mark.parametrize("offs", [(0, 0), (3, 3), (0, 5), (9, 2)])
@pytest.mark.parametrize("npt", [(4, 4), (8, 5), (16, 16), (1, 1)])
def test_confusion_counts(torch_dev, n, offs, npt):
    torch, d = torch_dev
    from paper_1601_00072_amd import confusion
    announce("confusion n", n, "offsets", offs, "classes", npt)
    rng = np.random.default_rng(n * 31 + offs[0] * 7 + offs[1] + npt[0])
    # mostly in range, a few out of range on either side
    pred = rng.integers(0, npt[0] + 1, n).astype(np.uint8)
    truth = rng.integers(0, npt[1] + 1, n).astype(np.uint8)
    pred[rng.random(n) < 0.01] = 255
    c = confusion(on_device(torch, d, pred, offs[0]), on_device(torch, d, truth, offs[1]), *npt)
    assert np.array_equal(c.cpu().numpy(), odice.confusion(pred, truth, *npt))


def test_empty_input(torch_dev):
    torch, d = torch_dev
    from paper_1601_00072_amd import confusion, dice
    announce("confusion empty")
    e = torch.empty(0, dtype=torch.uint8, device=d)
    c = confusion(e, e, 4, 4)
    assert np.all(c.cpu().numpy() == 0)
    assert np.all(np.isnan(dice(c, 4, 4).cpu().numpy()))


@pytest.mark.parametrize("class_of", [None, [3, 0, 2, 1], [1, -1, 0, 1], [-1, -1, -1, -1]])
def test_dice_exact(torch_dev, class_of):
    torch, d = torch_dev
    from paper_1601_00072_amd import confusion, dice
    announce("dice class_of", class_of)
    rng = np.random.default_rng(5)
    n = 300_001
    truth = rng.integers(0, 4, n).astype(np.uint8)
    pred = np.where(rng.random(n) < 0.7, truth, rng.integers(0, 4, n)).astype(np.uint8)
    truth[:40] = 3  # class 3 present; class 2 absent from pred where class_of says so
    got = dice(confusion(on_device(torch, d, pred, 0), on_device(torch, d, truth, 0), 4, 4), 4, 4, class_of)
    ref = odice.dsc(pred, truth, class_of if class_of is not None else [0, 1, 2, 3], 4)
    got = got.cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(got[~np.isnan(ref)], ref[~np.isnan(ref)])


@pytest.mark.parametrize("shape,seed", [((64, 128, 128), 2), ((256, 256), 1), ((40, 96, 96), 8)])
def test_phantom_segmentation_dice(torch_dev, shape, seed):
    """Dice of the GPU segmentation against the phantom's tissue labels equals
    the Dice of the oracle's segmentation (the labels agree bit for bit)."""
    torch, d = torch_dev
    from paper_1601_00072_amd import FCM, confusion, dice, rank_classes
    announce("phantom dice", shape, seed)
    img, lab = phantom(PhantomParams(shape=shape, seed=seed), with_labels=True)
    x = torch.from_numpy(img.ravel()).to(d)
    with FCM(x, 4) as f:
        r = f.solve()
        labels = f.labels()
    cls = rank_classes(r.centroids, 4)
    got = dice(confusion(labels, torch.from_numpy(lab.ravel()).to(d), 4, 4), 4, 4, cls).cpu().numpy()
    glab = labels.cpu().numpy()
    # the kernels: bit-exact on the GPU's own labels
    assert np.array_equal(got, odice.dsc(glab, lab, odice.rank_classes(r.centroids, 4), 4))
    # the segmentation: the oracle's labels and tissue map give the same scores
    ora = fcm_ref.solve(img, 4, 2.0, 1e-5, 300)
    vT = ora.v[ora.T]
    assert cls == odice.rank_classes(vT, 4)
    amb = P.check_labels(img, glab, vT)
    ref = odice.dsc(fcm_ref.defuzzify(img, vT), lab, odice.rank_classes(vT, 4), 4)
    if amb == 0:
        assert np.array_equal(got, ref), (got, ref)
    else:
        assert np.allclose(got, ref, rtol=0, atol=1e-3), (got, ref)
    assert np.all(got > 0.5)


def test_large_volume_counts(torch_dev):
    torch, d = torch_dev
    from paper_1601_00072_amd import FCM, confusion
    announce("confusion 512x512x256")
    img, lab = phantom(PhantomParams(shape=(256, 512, 512), seed=3, sigma=9.0, bias=0.2), with_labels=True)
    x = torch.from_numpy(img.ravel()).to(d)
    with FCM(x, 4) as f:
        f.solve()
        labels = f.labels()
    c = confusion(labels, torch.from_numpy(lab.ravel()).to(d), 4, 4).cpu().numpy()
    assert np.array_equal(c, odice.confusion(labels.cpu().numpy(), lab, 4, 4))
