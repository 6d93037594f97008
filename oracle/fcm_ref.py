"""Literal FP64 Fuzzy C-Means (test infrastructure only; see package docstring).

Follows Sec. 2.1 of the paper: objective Eq.1, constraints Eq.2, centroid
update Eq.3, membership update Eq.4, iterated as in Algorithm 1, on the grey
level of each pixel/voxel as the single feature.

Readings of points the paper leaves open (listed with the rest in the design
notes):
  * Eq.3 is printed with v_i and Eq.1 is labelled J_i; read as v_j and J_m.
  * m must exceed 1 (the exponent 2/(m-1) is undefined at m = 1).
  * Initialisation, default: centroid-first, v^0 is given (evenly spaced
    over [min, max] including both ends, computed in FP64 and rounded to FP32),
    then U^0 = memb(v^0).  The paper's own protocol (``solve_random_u``):
    U^0 random (positive weights per voxel normalised to sum 1, Eq.2), then
    the centroids first.
  * Stopping test: max_{i,j} |u_ij^t - u_ij^(t-1)| < eps, strict.
  * Zero distance (Eq.4 divides by zero): the membership is split equally
    over the clusters at distance 0 (membership 1 when only one is).
  * Empty cluster (sum of u^m is 0): the centroid keeps its previous value.
  * Defuzzification: the cluster of maximal membership; ties go to the lowest
    index.  For m > 1 that is the nearest centroid, evaluated in FP64.
  * The result is v^T, the centroids that produced the converged U^T.
"""
from __future__ import annotations

import dataclasses

import numpy as np

OK = 0
NOT_CONVERGED = 1


def linspace_init(lo: int, hi: int, C: int) -> np.ndarray:
    """Evenly spaced initial centroids over [lo, hi]: v_j = lo + j*(hi-lo)/(C-1)
    evaluated in FP64 (the quotient correctly rounded), then rounded to FP32.
    Returned as FP64 holding the FP32 values."""
    v = [float(lo) + (j * (int(hi) - int(lo))) / (C - 1) for j in range(C)]
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def memberships(x: np.ndarray, v: np.ndarray, m: float) -> np.ndarray:
    """Eq.4 as printed: u_ij = 1 / sum_k (d_ij / d_ik)^(2/(m-1)), d_ij = |x_i - v_j|.

    O(C^2) per voxel, exactly the double sum of the equation.  Rows with a zero
    distance take the equal split over their zero-distance clusters."""
    x = np.asarray(x, dtype=np.float64).ravel()
    v = np.asarray(v, dtype=np.float64)
    C = v.shape[0]
    e = 2.0 / (m - 1.0)
    d = np.abs(x[:, None] - v[None, :])
    zero = d == 0.0
    nz = zero.sum(axis=1)
    regular = nz == 0
    U = np.zeros((x.shape[0], C), dtype=np.float64)
    dr = d[regular]
    for j in range(C):
        s = np.zeros(dr.shape[0], dtype=np.float64)
        for k in range(C):
            s += (dr[:, j] / dr[:, k]) ** e
        U[regular, j] = 1.0 / s
    if not regular.all():
        sing = ~regular
        U[sing] = zero[sing] / nz[sing][:, None]
    return U


def centroids(x: np.ndarray, U: np.ndarray, m: float, v_prev: np.ndarray) -> np.ndarray:
    """Eq.3: v_j = sum_i u_ij^m x_i / sum_i u_ij^m (keep v_prev[j] if the denominator is 0)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    a = U ** m
    num = (a * x[:, None]).sum(axis=0)
    den = a.sum(axis=0)
    v = np.array(v_prev, dtype=np.float64, copy=True)
    ok = den > 0.0
    v[ok] = num[ok] / den[ok]
    return v


def objective(x: np.ndarray, U: np.ndarray, v: np.ndarray, m: float) -> float:
    """Eq.1: J_m = sum_i sum_j u_ij^m ||x_i - v_j||^2."""
    x = np.asarray(x, dtype=np.float64).ravel()
    return float(((U ** m) * (x[:, None] - np.asarray(v)[None, :]) ** 2).sum())


def defuzzify(x: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Label of maximal membership, i.e. the nearest centroid for m > 1; ties to the
    lowest index (np.argmin returns the first minimum)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    d = np.abs(x[:, None] - np.asarray(v, dtype=np.float64)[None, :])
    return np.argmin(d, axis=1).astype(np.uint8)


@dataclasses.dataclass
class Trajectory:
    v: list            # v[t] for t = 0..T (FP64 arrays of length C)
    delta: list        # delta[t] for t = 0..T (delta[0] is nan: no previous U)
    J: list            # J[t] = J_m(U^t, v^t) for t = 0..T
    T: int             # iterations performed
    status: int        # OK or NOT_CONVERGED

    @property
    def centroids(self) -> np.ndarray:
        return self.v[self.T]


def solve(x: np.ndarray, C: int, m: float = 2.0, eps: float = 1e-5, max_iter: int = 300,
          v0: np.ndarray | None = None) -> Trajectory:
    """Algorithm 1 with centroid-first initialisation.

    U^0 = memb(v^0); for t = 1..max_iter: v^t = cent(U^(t-1)), U^t = memb(v^t),
    delta^t = max |U^t - U^(t-1)|; stop with T = t when delta^t < eps."""
    x = np.asarray(x).ravel()
    if v0 is None:
        v0 = linspace_init(int(x.min()), int(x.max()), C)
    v = np.asarray(v0, dtype=np.float64).copy()
    U = memberships(x, v, m)
    vs, ds, Js = [v.copy()], [float("nan")], [objective(x, U, v, m)]
    status, T = NOT_CONVERGED, max_iter
    for t in range(1, max_iter + 1):
        v = centroids(x, U, m, v)
        U_new = memberships(x, v, m)
        delta = float(np.max(np.abs(U_new - U)))
        U = U_new
        vs.append(v.copy())
        ds.append(delta)
        Js.append(objective(x, U, v, m))
        if delta < eps:
            status, T = OK, t
            break
    return Trajectory(v=vs, delta=ds, J=Js, T=T, status=status)


def random_memberships(r: np.ndarray) -> np.ndarray:
    """U^0 from positive random weights r [n][C]: each row divided by its sum,
    so that Eq.2 holds."""
    r = np.asarray(r, dtype=np.float64)
    return r / r.sum(axis=1, keepdims=True)


def solve_random_u(x: np.ndarray, C: int, m: float, eps: float, max_iter: int, r: np.ndarray) -> Trajectory:
    """Algorithm 1 as the paper runs it: U^0 random (from the weights r, see
    random_memberships), then for t = 1..max_iter: v^t = cent(U^(t-1)) (Eq.3),
    U^t = memb(v^t) (Eq.4), delta^t = max |U^t - U^(t-1)|; stop with T = t
    when delta^t < eps.  No centroids exist before the first update, so v[0],
    delta[0] and J[0] are NaN; the result is v^T as in ``solve``."""
    x = np.asarray(x).ravel()
    U = random_memberships(r)
    assert U.shape == (x.size, C)
    v = np.full(C, np.nan)
    vs, ds, Js = [v.copy()], [float("nan")], [float("nan")]
    status, T = NOT_CONVERGED, max_iter
    for t in range(1, max_iter + 1):
        v = centroids(x, U, m, v)
        U_new = memberships(x, v, m)
        delta = float(np.max(np.abs(U_new - U)))
        U = U_new
        vs.append(v.copy())
        ds.append(delta)
        Js.append(objective(x, U, v, m))
        if delta < eps:
            status, T = OK, t
            break
    return Trajectory(v=vs, delta=ds, J=Js, T=T, status=status)
