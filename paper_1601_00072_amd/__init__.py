"""gfx950 Fuzzy C-Means segmentation (arXiv 1601.00072), Python binding of libfcm.so.

PyTorch supplies device memory and streams; every step of the iteration runs
in the library's HIP kernels.
"""
from .api import FCM, MLP, FCMBatch, FcmError, Result, confusion, dice, histogram, paper_baseline, rank_classes, solve

__all__ = ["FCM", "FCMBatch", "MLP", "FcmError", "Result", "confusion", "dice", "histogram", "paper_baseline", "rank_classes", "solve"]
