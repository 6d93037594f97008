"""Oracle-F: the FP64 per-voxel oracle in C, threaded over the host cores.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Computes what
``fcm_ref.solve`` computes (Algorithm 1, centroid-first start, Eq.4 in the
w / sum w form), in plain C with one static chunk of voxels per thread and the
chunk sums added in thread order.  Used for the CPU timing leg of the
benchmark and for sizes where the numpy literal oracle is slow.  Pinned
against the literal oracle in tests/test_oracle_fast.py.  The shared library
is compiled from fcm_fast.c with gcc on first use (or by the build step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .fcm_ref import NOT_CONVERGED, OK, Trajectory, linspace_init

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fcm_fast.c")
LIB = os.path.join(HERE, "_build", "liboracle_f.so")
_lib = None


def build() -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_f_solve.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, ctypes.POINTER(ctypes.c_int)]
        lib.oracle_f_solve.restype = ctypes.c_int
        _lib = lib
    return _lib


def solve(x: np.ndarray, C: int, m: float = 2.0, eps: float = 1e-5, max_iter: int = 300,
          v0: np.ndarray | None = None, threads: int = 0) -> Trajectory:
    """Same result as fcm_ref.solve (up to summation order); threads < 1 uses
    every host core."""
    lib = _load()
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint8).ravel())
    if v0 is None:
        v0 = linspace_init(int(x.min()), int(x.max()), C)
    v0 = np.ascontiguousarray(np.asarray(v0, dtype=np.float64))
    vh = np.zeros((max_iter + 1, C))
    dh = np.zeros(max_iter + 1)
    Jh = np.zeros(max_iter + 1)
    st = ctypes.c_int()
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    T = lib.oracle_f_solve(x.ctypes.data, x.size, int(C), float(m), float(eps), int(max_iter), dp(v0), int(threads),
                           dp(vh), dp(dh), dp(Jh), ctypes.byref(st))
    if T < 0:
        raise ValueError("invalid arguments")
    return Trajectory(v=[vh[t].copy() for t in range(T + 1)], delta=[float(d) for d in dh[:T + 1]],
                      J=[float(j) for j in Jh[:T + 1]], T=int(T), status=OK if st.value == 0 else NOT_CONVERGED)
