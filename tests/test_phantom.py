"""The seeded input generator: determinism, structure and value distribution (CPU)."""
import json
import os

import numpy as np
import pytest

from phantom import PhantomParams, batch_instances, jittered_params, phantom, sha256, uniform01

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_hashes():
    with open(os.path.join(GOLDEN, "phantom_hashes.json")) as f:
        cases = json.load(f)
    for name, c in cases.items():
        p = PhantomParams(shape=tuple(c["shape"]), seed=c["seed"], sigma=c["sigma"], bias=c["bias"])
        img, lab = phantom(p, with_labels=True)
        assert sha256(img) == c["image_sha256"], name
        assert sha256(lab) == c["labels_sha256"], name


def test_chunking_does_not_change_bytes():
    p = PhantomParams(shape=(9, 31, 37), seed=11)
    a = phantom(p, chunk_voxels=1 << 22)
    b = phantom(p, chunk_voxels=37 * 5)
    assert np.array_equal(a, b)


def test_structure_and_means():
    img, lab = phantom(PhantomParams(shape=(256, 256), seed=3, bias=0.0), with_labels=True)
    assert img.dtype == np.uint8
    counts = np.bincount(lab.ravel(), minlength=4)
    assert np.all(counts > 1000)
    # nested: WM core at the centre, background in the corner
    assert lab[128, 128] == 3 and lab[0, 0] == 0
    # class means within noise of 0/40/110/150 (background clipped at 0)
    for k, mu in ((1, 40), (2, 110), (3, 150)):
        assert abs(img[lab == k].mean() - mu) < 1.0
    assert abs(img[lab == 1].std() - 8.0) < 0.5


def test_uniform_stream_properties():
    u = uniform01(1234, np.arange(200000))
    assert 0.0 < u.min() and u.max() <= 1.0
    assert abs(u.mean() - 0.5) < 0.005


def test_jitter_and_batch_lists():
    p = jittered_params((256, 256), seed=10**6 + 3)
    assert list(p.means) == sorted(p.means) and p.means[0] == 0.0
    assert 3.0 <= p.sigma <= 10.0 and 0.0 <= p.bias <= 0.2
    inst = batch_instances()
    assert len(inst) == 512
    sizes = [int(np.prod(q.shape)) for q, _ in inst]
    assert min(sizes) >= 64 * 64 and max(sizes) <= 160 ** 3
    assert all(3 <= c <= 8 for _, c in inst)
    assert 60e6 < sum(sizes) < 110e6
