"""Pins of the Dice oracle (Eq.5) against hand-counted cases and identities
that do not go through its formula."""
import numpy as np
import pytest

from oracle import dice


def test_hand_counted_example():
    # truth: class 1 at voxels {0,1,2}, class 0 at {3,4,5}
    # pred:  cluster 1 at {0,1,5}, cluster 0 at {2,3,4}
    truth = np.array([1, 1, 1, 0, 0, 0], np.uint8)
    pred = np.array([1, 1, 0, 0, 0, 1], np.uint8)
    # class 1: |PR and GT| = |{0,1}| = 2, |PR| = 3, |GT| = 3 -> 4/6
    # class 0: |{3,4}| = 2, 3, 3 -> 4/6
    got = dice.dsc(pred, truth, [0, 1], 2)
    assert got[0] == 4 / 6 and got[1] == 4 / 6
    # clusters swapped in meaning: class 0 = {0,1,5} vs {3,4,5}: |{5}| = 1 -> 2/6
    got = dice.dsc(pred, truth, [1, 0], 2)
    assert got[0] == 2 / 6 and got[1] == 2 / 6


def test_identical_disjoint_and_empty():
    rng = np.random.default_rng(0)
    t = rng.integers(0, 4, 1000).astype(np.uint8)
    assert np.all(dice.dsc(t, t, [0, 1, 2, 3], 4) == 1.0)
    # every voxel moved to the next class: no overlap anywhere
    assert np.all(dice.dsc((t + 1) % 4, t, [0, 1, 2, 3], 4) == 0.0)
    # class 3 absent from both: 0/0
    t3 = np.minimum(t, 2)
    d = dice.dsc(t3, t3, [0, 1, 2, 3], 4)
    assert np.all(d[:3] == 1.0) and np.isnan(d[3])
    # class present in truth only
    d = dice.dsc(np.zeros(5, np.uint8), np.array([0, 0, 0, 1, 1], np.uint8), [0, 1], 2)
    assert d[1] == 0.0 and d[0] == 2 * 3 / (5 + 3)


def test_jaccard_identity_by_python_sets():
    """DSC = 2 J / (1 + J) with J = |A and B| / |A or B| counted on Python sets."""
    rng = np.random.default_rng(7)
    truth = rng.integers(0, 4, 3000).astype(np.uint8)
    pred = np.where(rng.random(3000) < 0.8, truth, rng.integers(0, 5, 3000)).astype(np.uint8)
    cls = [2, 0, 3, 1, -1]
    d = dice.dsc(pred, truth, cls, 4)
    for k in range(4):
        a = {i for i in range(3000) if pred[i] < len(cls) and cls[pred[i]] == k}
        b = {i for i in range(3000) if truth[i] == k}
        jac = len(a & b) / len(a | b)
        assert d[k] == pytest.approx(2 * jac / (1 + jac), rel=1e-14)


def test_symmetric_and_permutation_invariant():
    rng = np.random.default_rng(3)
    truth = rng.integers(0, 3, 2000).astype(np.uint8)
    pred = rng.integers(0, 3, 2000).astype(np.uint8)
    a = dice.dsc(pred, truth, [0, 1, 2], 3)
    b = dice.dsc(truth, pred, [0, 1, 2], 3)
    assert np.array_equal(a, b)
    perm = np.array([2, 0, 1])
    # renaming clusters, with the map renamed alike, changes nothing
    pred2 = perm[pred].astype(np.uint8)
    cls2 = [0] * 3
    for j in range(3):
        cls2[perm[j]] = j
    assert np.array_equal(dice.dsc(pred2, truth, cls2, 3), a)


def test_confusion_margins():
    rng = np.random.default_rng(11)
    truth = rng.integers(0, 6, 5000).astype(np.uint8)
    pred = rng.integers(0, 9, 5000).astype(np.uint8)
    c = dice.confusion(pred, truth, 8, 5)
    m = c[:-1].reshape(8, 5)
    inside = (pred < 8) & (truth < 5)
    assert c.sum() == 5000
    assert c[-1] == np.count_nonzero(~inside)
    assert np.array_equal(m.sum(axis=1), np.bincount(pred[inside], minlength=8)[:8])
    assert np.array_equal(m.sum(axis=0), np.bincount(truth[inside], minlength=5)[:5])
    # brute force on a few cells
    for j, k in [(0, 0), (3, 4), (7, 2)]:
        assert m[j, k] == sum(1 for i in range(5000) if pred[i] == j and truth[i] == k)


def test_rank_classes():
    assert dice.rank_classes([150.0, 2.0, 110.0, 40.0], 4) == [3, 0, 2, 1]
    assert dice.rank_classes([5.0, 5.0, 1.0], 2) == [1, -1, 0]
