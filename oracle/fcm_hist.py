"""FP64 Fuzzy C-Means regrouped over the 256 grey levels (test infrastructure only).

For 8-bit data every per-voxel quantity of Sec. 2.1 depends on the voxel only
through its grey level g, so each sum over voxels in Eq.1 and Eq.3 equals
sum_g h_g f(g) with h the grey-level histogram; the maximum over voxels in the
stopping test equals the maximum over the levels that occur (h_g > 0).  This
is the data-reduction idea behind brFCM (Sec. 3).  The regrouping changes only
the rounding order, so this module must agree with ``fcm_ref`` to rounding,
which the tests check; it lets the large and batched workloads be checked at
full size.

Memberships are written here in the normalised-weight form
u_ij = w_ij / sum_k w_ik with w_ij = d_ij^(-2/(m-1)), algebraically equal to
Eq.4, so that agreement with the literal module also cross-checks the form.
"""
from __future__ import annotations

import numpy as np

from .fcm_ref import NOT_CONVERGED, OK, Trajectory, linspace_init

LEVELS = np.arange(256, dtype=np.float64)


def histogram(x: np.ndarray) -> np.ndarray:
    return np.bincount(np.asarray(x, dtype=np.uint8).ravel(), minlength=256).astype(np.int64)


def level_memberships(g: np.ndarray, v: np.ndarray, m: float) -> np.ndarray:
    d = np.abs(g[:, None] - np.asarray(v, dtype=np.float64)[None, :])
    zero = d == 0.0
    nz = zero.sum(axis=1)
    U = np.empty_like(d)
    reg = nz == 0
    w = d[reg] ** (-2.0 / (m - 1.0))
    U[reg] = w / w.sum(axis=1, keepdims=True)
    U[~reg] = zero[~reg] / nz[~reg][:, None]
    return U


def solve(hist: np.ndarray, C: int, m: float = 2.0, eps: float = 1e-5, max_iter: int = 300,
          v0: np.ndarray | None = None) -> Trajectory:
    hist = np.asarray(hist, dtype=np.int64)
    present = np.nonzero(hist)[0]
    g = LEVELS[present]
    h = hist[present].astype(np.float64)
    if v0 is None:
        v0 = linspace_init(int(present.min()), int(present.max()), C)
    v = np.asarray(v0, dtype=np.float64).copy()

    def J(U, v):
        return float((h[:, None] * U ** m * (g[:, None] - v[None, :]) ** 2).sum())

    U = level_memberships(g, v, m)
    vs, ds, Js = [v.copy()], [float("nan")], [J(U, v)]
    status, T = NOT_CONVERGED, max_iter
    for t in range(1, max_iter + 1):
        a = h[:, None] * U ** m
        num = (a * g[:, None]).sum(axis=0)
        den = a.sum(axis=0)
        v = v.copy()
        ok = den > 0.0
        v[ok] = num[ok] / den[ok]
        U_new = level_memberships(g, v, m)
        delta = float(np.max(np.abs(U_new - U)))
        U = U_new
        vs.append(v.copy())
        ds.append(delta)
        Js.append(J(U, v))
        if delta < eps:
            status, T = OK, t
            break
    return Trajectory(v=vs, delta=ds, J=Js, T=T, status=status)


def level_labels(v: np.ndarray) -> np.ndarray:
    """Nearest-centroid label of each grey level (FP64, ties to the lowest index)."""
    d = np.abs(LEVELS[:, None] - np.asarray(v, dtype=np.float64)[None, :])
    return np.argmin(d, axis=1).astype(np.uint8)
