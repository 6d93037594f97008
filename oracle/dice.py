"""Dice similarity coefficient per tissue class (Sec. 5.2.2, Eq.5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq.5 compares the set PR of voxels a segmentation assigns to a tissue with
the set GT of voxels of that tissue in the ground truth:
DSC = 2 |PR and GT| / (|PR| + |GT|).  A segmentation labels voxels by cluster
index; ``class_of[j]`` names the tissue that cluster j stands for (-1: none).
Where both sets are empty the ratio is 0/0 and is reported as NaN (the paper
does not meet that case).  Parity pinned by tests/test_dice_ref.py.
"""
from __future__ import annotations

import numpy as np


def class_sets(pred: np.ndarray, truth: np.ndarray, class_of, k: int):
    """Boolean masks PR_k (voxels whose cluster stands for class k) and GT_k."""
    pred = np.asarray(pred).ravel()
    truth = np.asarray(truth).ravel()
    lut = np.asarray(list(class_of), dtype=np.int64)
    mapped = np.full(pred.shape, -1, dtype=np.int64)
    ok = pred < lut.size
    mapped[ok] = lut[pred[ok]]
    return mapped == k, truth == k


def dsc(pred: np.ndarray, truth: np.ndarray, class_of, n_classes: int) -> np.ndarray:
    """Eq.5 for every class 0..n_classes-1, from the two sets' sizes."""
    out = np.empty(n_classes, dtype=np.float64)
    for k in range(n_classes):
        pr, gt = class_sets(pred, truth, class_of, k)
        inter = int(np.count_nonzero(pr & gt))
        den = int(np.count_nonzero(pr)) + int(np.count_nonzero(gt))
        out[k] = (2 * inter) / den if den else np.nan
    return out


def confusion(pred: np.ndarray, truth: np.ndarray, n_pred: int, n_truth: int) -> np.ndarray:
    """counts[j * n_truth + k] = |pred == j and truth == k|; the last entry
    counts voxels with pred >= n_pred or truth >= n_truth."""
    pred = np.asarray(pred).ravel().astype(np.int64)
    truth = np.asarray(truth).ravel().astype(np.int64)
    out = np.zeros(n_pred * n_truth + 1, dtype=np.int64)
    for j in range(n_pred):
        pj = pred == j
        for k in range(n_truth):
            out[j * n_truth + k] = np.count_nonzero(pj & (truth == k))
    out[-1] = np.count_nonzero((pred >= n_pred) | (truth >= n_truth))
    return out


def rank_classes(centroids, n_classes: int):
    """The cluster with the r-th smallest centroid stands for class r (classes
    numbered by increasing mean intensity); ties by cluster index."""
    v = np.asarray(centroids, dtype=np.float64)
    order = np.lexsort((np.arange(v.size), v))
    out = [-1] * v.size
    for r, j in enumerate(order):
        if r < n_classes:
            out[int(j)] = r
    return out
