"""Python face of the C ABI: one ``FCM`` object per solver handle."""
from __future__ import annotations

import ctypes
import dataclasses
import os
import sys

import numpy as np

from . import _lib as L


class FcmError(RuntimeError):
    def __init__(self, status: int, what: str):
        lib = L.load()
        msg = lib.fcm_strerror(status).decode()
        detail = lib.fcm_last_error().decode() if status == L.FCM_EDEVICE else ""
        super().__init__(f"{what}: {msg} ({status}){' -- ' + detail if detail else ''}")
        self.status = status


@dataclasses.dataclass
class Result:
    iters: int
    passes: int
    status: int
    delta: float
    J: float
    centroids: np.ndarray
    kernel_ms: float
    lo: int
    hi: int

    @property
    def converged(self) -> bool:
        return self.status == L.FCM_OK


def _result(r: L.FcmResult) -> Result:
    C = r.n_clusters
    return Result(iters=r.iters, passes=r.passes, status=r.status, delta=r.delta, J=r.J,
                  centroids=np.array(r.centroids[:C], dtype=np.float64), kernel_ms=r.kernel_ms,
                  lo=r.lo, hi=r.hi)


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


class FCM:
    """Fuzzy C-Means solver over a uint8 device tensor (any shape, contiguous).

    ``init`` is None (evenly spaced over the data range), a sequence of C
    starting centroids, or ``("random_u", seed)`` for the paper's own start
    (random memberships from the SplitMix64 stream ``seed``, centroids first).  The tensor is borrowed: keep it alive and unmodified
    while the solver exists."""

    def __init__(self, x, n_clusters: int, m: float = 2.0, eps: float = 1e-5, max_iter: int = 300,
                 init=None, kahan_only: bool = False, timing: bool = False, stream=None):
        import torch
        if not isinstance(x, torch.Tensor) or x.dtype != torch.uint8 or not x.is_cuda:
            raise TypeError("x must be a uint8 CUDA/HIP tensor")
        if not x.is_contiguous():
            raise ValueError("x must be contiguous")
        self._lib = L.load()
        self.x = x
        self.n = x.numel()
        self.C = int(n_clusters)
        self._stream = stream if stream is not None else torch.cuda.current_stream(x.device)
        flags = (L.FCM_F_KAHAN_ONLY if kahan_only else 0) | (L.FCM_F_TIMING if timing else 0)
        self._init_buf = None
        seed = 0
        if init is None:
            mode, ptr = L.FCM_INIT_LINSPACE, None
        elif isinstance(init, tuple) and len(init) == 2 and init[0] == "random_u":
            mode, ptr, seed = L.FCM_INIT_RANDOM_U, None, int(init[1]) & ((1 << 64) - 1)
        else:
            v = np.ascontiguousarray(np.asarray(init, dtype=np.float64))
            if v.shape != (self.C,):
                raise ValueError("init must hold n_clusters values")
            self._init_buf = (ctypes.c_double * self.C)(*v.tolist())
            mode, ptr = L.FCM_INIT_GIVEN, ctypes.cast(self._init_buf, ctypes.POINTER(ctypes.c_double))
        p = L.FcmParams(n_clusters=self.C, m=float(m), eps=float(eps), max_iter=int(max_iter), init=mode,
                        init_centroids=ptr, flags=flags, seed=seed)
        self._h = ctypes.c_void_p()
        rc = self._lib.fcm_init(ctypes.byref(self._h), ctypes.c_void_p(x.data_ptr()), self.n, ctypes.byref(p),
                                ctypes.c_void_p(self._stream.cuda_stream))
        if rc != L.FCM_OK:
            self._h = None
            raise FcmError(rc, "fcm_init")

    # -- tuning ---------------------------------------------------------------
    @property
    def tuning(self) -> dict:
        t = L.FcmTuning()
        self._check(self._lib.fcm_get_tuning(self._h, ctypes.byref(t)), "fcm_get_tuning")
        return {f: getattr(t, f) for f, _ in L.FcmTuning._fields_}

    def set_tuning(self, **kw):
        cur = self.tuning
        cur.update(kw)
        if "grid" not in kw:
            cur["grid"] = 0
        t = L.FcmTuning(**cur)
        self._check(self._lib.fcm_set_tuning(self._h, ctypes.byref(t)), "fcm_set_tuning")

    def autotune(self, cache: str | None = None, reps: int = 3):
        """Time candidate launch configurations on this input and keep the
        fastest that agrees with the current one (see fcm_autotune).
        Returns (tuning dict, median ms per solve)."""
        t, ms = L.FcmTuning(), ctypes.c_double()
        self._check(self._lib.fcm_autotune(self._h, None if cache is None else str(cache).encode(), int(reps),
                                           ctypes.byref(t), ctypes.byref(ms)), "fcm_autotune")
        return {f: getattr(t, f) for f, _ in L.FcmTuning._fields_}, ms.value

    def set_wait_limit(self, seconds: float = 0.0) -> int:
        """Set the wall-clock limit of one cross-block wait (0 keeps it);
        returns how many solves were run again in a cooperative launch after
        a resident launch gave up (fcm_set_wait_limit)."""
        rec = ctypes.c_int32()
        self._check(self._lib.fcm_set_wait_limit(self._h, float(seconds), ctypes.byref(rec)), "fcm_set_wait_limit")
        return rec.value

    # -- iteration --------------------------------------------------------------
    def reset(self):
        """Restart from v^0 on the same (possibly rewritten) input; no allocation."""
        self._check(self._lib.fcm_reset(self._h), "fcm_reset")

    def iterate(self, k: int) -> Result:
        r = L.FcmResult()
        rc = self._lib.fcm_iterate(self._h, int(k), ctypes.byref(r))
        if rc < 0 and rc != L.FCM_ENUMERIC:
            raise FcmError(rc, "fcm_iterate")
        return _result(r)

    def solve(self) -> Result:
        r = L.FcmResult()
        rc = self._lib.fcm_solve(self._h, ctypes.byref(r))
        if rc < 0 and rc != L.FCM_ENUMERIC:
            raise FcmError(rc, "fcm_solve")
        return _result(r)

    def solve_async(self, labels=None):
        """Enqueue a whole solve without waiting (fcm_solve_async); with
        `labels` (a uint8 device tensor of the input's size) the same launch
        also writes the labels of the result.  Read the result with result()."""
        import torch
        ptr = None
        if labels is not None:
            if labels.dtype != torch.uint8 or not labels.is_cuda or labels.numel() != self.n or \
                    not labels.is_contiguous():
                raise ValueError("labels must be a contiguous uint8 device tensor of the input's size")
            ptr = ctypes.c_void_p(labels.data_ptr())
        self._check(self._lib.fcm_solve_async(self._h, ptr), "fcm_solve_async")

    def result(self):
        """Wait and report the last solve (fcm_solve_wait); returns (Result, fused
        passes committed on this handle so far)."""
        r, tot = L.FcmResult(), ctypes.c_int64()
        rc = self._lib.fcm_solve_wait(self._h, ctypes.byref(r), ctypes.byref(tot))
        if rc < 0 and rc != L.FCM_ENUMERIC:
            raise FcmError(rc, "fcm_solve_wait")
        return _result(r), int(tot.value)

    def labels(self, out=None):
        import torch
        if out is None:
            out = torch.empty_like(self.x)
        if out.dtype != torch.uint8 or not out.is_cuda or out.numel() != self.n or not out.is_contiguous():
            raise ValueError("out must be a contiguous uint8 device tensor of the input's size")
        self._check(self._lib.fcm_labels(self._h, ctypes.c_void_p(out.data_ptr())), "fcm_labels")
        return out

    def centroids(self) -> np.ndarray:
        buf = (ctypes.c_double * self.C)()
        self._check(self._lib.fcm_centroids(self._h, buf), "fcm_centroids")
        return np.array(buf[:], dtype=np.float64)

    def trajectory(self, t: int):
        v = (ctypes.c_double * self.C)()
        d, J = ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.fcm_trajectory(self._h, int(t), v, ctypes.byref(d), ctypes.byref(J)),
                    "fcm_trajectory")
        return np.array(v[:], dtype=np.float64), d.value, J.value

    def solve_warm(self, net: "MLP", check: bool = False):
        """Solve from the network's start centroids (histogram -> BF16 network
        -> start).  check: also solve from the handle's own start and keep the
        warm result only if its J is within 1e-6 (relative) of the plain one,
        else fall back.  Returns (result, used_warm, plain result or None)."""
        r, rp, used = L.FcmResult(), L.FcmResult(), ctypes.c_int32()
        rc = self._lib.fcm_solve_warm(self._h, net._h, 1 if check else 0, ctypes.byref(r), ctypes.byref(rp),
                                      ctypes.byref(used))
        if rc < 0 and rc != L.FCM_ENUMERIC:
            raise FcmError(rc, "fcm_solve_warm")
        return _result(r), bool(used.value), (_result(rp) if check else None)

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.fcm_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # at interpreter shutdown the HIP runtime (and any profiler attached
        # to it) may already be torn down: release nothing then
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if self._h is None:
            raise FcmError(L.FCM_ESTATE, what)
        if rc != L.FCM_OK:
            raise FcmError(rc, what)


def solve(x, n_clusters: int, m: float = 2.0, eps: float = 1e-5, max_iter: int = 300, init=None,
          kahan_only: bool = False, labels: bool = True):
    """One-shot solve: returns (Result, labels tensor or None)."""
    with FCM(x, n_clusters, m=m, eps=eps, max_iter=max_iter, init=init, kahan_only=kahan_only) as f:
        res = f.solve()
        lab = f.labels() if labels else None
        return res, lab


class FCMBatch:
    """Many instances solved in one persistent launch.

    ``x``: one contiguous uint8 device tensor holding the instances back to
    back; ``sizes``: voxel count of each instance; ``params``: one dict per
    instance with keys n_clusters (required), m, eps, max_iter, init,
    kahan_only."""

    def __init__(self, x, sizes, params, stream=None):
        import torch
        if not isinstance(x, torch.Tensor) or x.dtype != torch.uint8 or not x.is_cuda or not x.is_contiguous():
            raise TypeError("x must be a contiguous uint8 CUDA/HIP tensor")
        self._lib = L.load()
        self.x = x
        sizes = [int(s) for s in sizes]
        if len(sizes) != len(params):
            raise ValueError("one parameter record per instance")
        self.count = len(sizes)
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        if self.offsets[-1] != x.numel():
            raise ValueError("sizes must add up to x.numel()")
        self.C = [int(q["n_clusters"]) for q in params]
        self._keep = []
        recs = (L.FcmParams * self.count)()
        for i, q in enumerate(params):
            init = q.get("init")
            if init is None:
                mode, ptr = L.FCM_INIT_LINSPACE, None
            else:
                buf = (ctypes.c_double * self.C[i])(*[float(v) for v in init])
                self._keep.append(buf)
                mode, ptr = L.FCM_INIT_GIVEN, ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
            recs[i] = L.FcmParams(n_clusters=self.C[i], m=float(q.get("m", 2.0)), eps=float(q.get("eps", 1e-5)),
                                  max_iter=int(q.get("max_iter", 300)), init=mode, init_centroids=ptr,
                                  flags=L.FCM_F_KAHAN_ONLY if q.get("kahan_only") else 0)
        self._stream = stream if stream is not None else torch.cuda.current_stream(x.device)
        off = self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        self._h = ctypes.c_void_p()
        rc = self._lib.fcm_batch_init(ctypes.byref(self._h), ctypes.c_void_p(x.data_ptr()), off, self.count, recs,
                                      ctypes.c_void_p(self._stream.cuda_stream))
        if rc != L.FCM_OK:
            self._h = None
            raise FcmError(rc, "fcm_batch_init")

    def set_tiling(self, chunks_per_thread: int = 4, grid: int = 0):
        rc = self._lib.fcm_batch_set_tiling(self._h, int(chunks_per_thread), int(grid))
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_set_tiling")

    def set_block(self, threads: int = 512):
        """Threads per block of the batched kernel: 128, 256 or 512 (fcm_batch_set_block)."""
        rc = self._lib.fcm_batch_set_block(self._h, int(threads))
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_set_block")

    def set_tail_tiling(self, from_pass: int = 96, chunks_per_thread: int = 2):
        """Finer tiles from pass `from_pass` on (fcm_batch_set_tail_tiling)."""
        rc = self._lib.fcm_batch_set_tail_tiling(self._h, int(from_pass), int(chunks_per_thread))
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_set_tail_tiling")

    def solve(self):
        out = (L.FcmResult * self.count)()
        rc = self._lib.fcm_batch_solve(self._h, out)
        if rc < 0 and rc != L.FCM_ENUMERIC:
            raise FcmError(rc, "fcm_batch_solve")
        return [_result(r) for r in out]

    def autotune(self, cache: str | None = None, reps: int = 2):
        """Pick the block size, tile size and grid (see fcm_batch_autotune);
        returns (block, chunks_per_thread, grid, median ms per batched solve)."""
        bs, cpt, grid, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        rc = self._lib.fcm_batch_autotune(self._h, None if cache is None else str(cache).encode(), int(reps),
                                          ctypes.byref(bs), ctypes.byref(cpt), ctypes.byref(grid), ctypes.byref(ms))
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_autotune")
        return bs.value, cpt.value, grid.value, ms.value

    def set_start(self, net: "MLP | None" = None, use=None):
        """Learned start for the instances whose C matches the network (and
        whose flag in `use` is set, if given); every other instance, or all
        with net=None, takes its own init."""
        flags = None
        if use is not None:
            buf = np.ascontiguousarray(np.asarray(use, dtype=np.uint8))
            if buf.shape != (self.count,):
                raise ValueError("one flag per instance")
            flags = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        rc = self._lib.fcm_batch_set_start(self._h, None if net is None else net._h, flags)
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_set_start")

    def solve_warm(self, net: "MLP", check: bool = True):
        """Warm-started batch solve with the fall-back rule per instance
        (fcm_batch_solve_warm).  Returns (results, used_warm flags, plain
        results or None); the batch keeps the starts of the returned results
        (set_start() goes back to each instance's own init)."""
        out = (L.FcmResult * self.count)()
        plain = (L.FcmResult * self.count)() if check else None
        used = (ctypes.c_uint8 * self.count)()
        rc = self._lib.fcm_batch_solve_warm(self._h, net._h, 1 if check else 0, out, plain, used)
        if rc < 0 and rc != L.FCM_ENUMERIC:
            raise FcmError(rc, "fcm_batch_solve_warm")
        return ([_result(r) for r in out], np.array(used[:], dtype=bool),
                None if plain is None else [_result(r) for r in plain])

    def targets(self, C: int, out=None):
        """Network training targets of the last solve (fcm_batch_targets):
        each instance's centroids sorted ascending, / 255, as a float32 device
        tensor [count, C]."""
        import torch
        if out is None:
            out = torch.empty((self.count, int(C)), dtype=torch.float32, device=self.x.device)
        if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != self.count * int(C):
            raise ValueError("out must be a contiguous float32 tensor of count * C values")
        rc = self._lib.fcm_batch_targets(self._h, int(C), ctypes.c_void_p(out.data_ptr()))
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_targets")
        return out

    def labels(self, out=None):
        import torch
        if out is None:
            out = torch.empty_like(self.x)
        rc = self._lib.fcm_batch_labels(self._h, ctypes.c_void_p(out.data_ptr()))
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_labels")
        return out

    def timeline(self, i: int):
        """Microseconds from the launch start until instance i committed its
        data range (entry 0) and each pass p (entry 1 + p) in the last solve
        (fcm_batch_timeline)."""
        cnt = ctypes.c_int32()
        rc = self._lib.fcm_batch_timeline(self._h, int(i), None, 0, ctypes.byref(cnt))
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_timeline")
        us = np.empty(cnt.value, dtype=np.float64)
        rc = self._lib.fcm_batch_timeline(self._h, int(i), us.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          cnt.value, None)
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_timeline")
        return us

    def trajectory(self, i: int, t: int):
        C = self.C[i]
        v = (ctypes.c_double * C)()
        d, J = ctypes.c_double(), ctypes.c_double()
        rc = self._lib.fcm_batch_trajectory(self._h, int(i), int(t), v, ctypes.byref(d), ctypes.byref(J))
        if rc != L.FCM_OK:
            raise FcmError(rc, "fcm_batch_trajectory")
        return np.array(v[:], dtype=np.float64), d.value, J.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fcm_batch_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # at interpreter shutdown the HIP runtime (and any profiler attached
        # to it) may already be torn down: release nothing then
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def histogram(x, sizes, stream=None):
    """Normalised 256-bin histograms of the instances packed back to back in
    the uint8 device tensor x; returns a float32 device tensor [count, 256]."""
    import torch
    lib = L.load()
    off = np.concatenate([[0], np.cumsum([int(v) for v in sizes])]).astype(np.int64)
    if off[-1] != x.numel():
        raise ValueError("sizes must add up to x.numel()")
    out = torch.empty((len(sizes), 256), dtype=torch.float32, device=x.device)
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    rc = lib.fcm_histogram(ctypes.c_void_p(x.data_ptr()), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           len(sizes), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream))
    if rc != L.FCM_OK:
        raise FcmError(rc, "fcm_histogram")
    return out


def paper_baseline(x, n_clusters: int, m: float = 2.0, eps: float = 0.005, max_iter: int = 300, init=None,
                   labels: bool = False, stream=None):
    """Solve with the paper's own GPU structure (fcm_paper_solve): per-cluster
    kernels, Algorithm 2 reductions, U copied to the host every iteration for
    the stopping test.  init: None (evenly spaced), C centroids, or
    ("random_u", seed).  Returns (Result, trajectory dict with "v" [T+1][C]
    and "delta" [T+1], host labels or None, stats dict)."""
    import torch
    lib = L.load()
    if not isinstance(x, torch.Tensor) or x.dtype != torch.uint8 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("x must be a contiguous uint8 device tensor")
    C = int(n_clusters)
    seed, ptr, keep = 0, None, None
    if init is None:
        mode = L.FCM_INIT_LINSPACE
    elif isinstance(init, tuple) and len(init) == 2 and init[0] == "random_u":
        mode, seed = L.FCM_INIT_RANDOM_U, int(init[1]) & ((1 << 64) - 1)
    else:
        v = [float(a) for a in init]
        if len(v) != C:
            raise ValueError("init must hold n_clusters values")
        keep = (ctypes.c_double * C)(*v)
        mode, ptr = L.FCM_INIT_GIVEN, ctypes.cast(keep, ctypes.POINTER(ctypes.c_double))
    p = L.FcmParams(n_clusters=C, m=float(m), eps=float(eps), max_iter=int(max_iter), init=mode,
                    init_centroids=ptr, flags=0, seed=seed)
    vh = np.full((int(max_iter) + 1, C), np.nan)
    dh = np.full(int(max_iter) + 1, np.nan)
    lab = np.empty(x.numel(), dtype=np.uint8) if labels else None
    r, st = L.FcmResult(), L.FcmPaperStats()
    rc = lib.fcm_paper_solve(ctypes.c_void_p(x.data_ptr()), x.numel(), ctypes.byref(p), _stream_handle(stream, x.device),
                             ctypes.byref(r), vh.ctypes.data_as(ctypes.c_void_p), dh.ctypes.data_as(ctypes.c_void_p),
                             None if lab is None else lab.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st))
    if rc < 0:
        raise FcmError(rc, "fcm_paper_solve")
    res = _result(r)
    traj = {"v": vh[:res.iters + 1], "delta": dh[:res.iters + 1]}
    stats = {f: getattr(st, f) for f, _ in L.FcmPaperStats._fields_}
    return res, traj, lab, stats


def confusion(pred, truth, n_pred: int, n_truth: int, stream=None):
    """Confusion counts of two uint8 label tensors on the device (Sec. 5.2.2):
    an int64 device tensor [n_pred * n_truth + 1]; entry j * n_truth + k counts
    voxels with pred j and truth k, the last one voxels outside the ranges."""
    import torch
    lib = L.load()
    if pred.dtype != torch.uint8 or truth.dtype != torch.uint8 or pred.numel() != truth.numel():
        raise ValueError("pred and truth must be uint8 tensors of equal size")
    if not (pred.is_contiguous() and truth.is_contiguous()):
        raise ValueError("pred and truth must be contiguous")
    out = torch.empty(int(n_pred) * int(n_truth) + 1, dtype=torch.int64, device=pred.device)
    st = stream if stream is not None else torch.cuda.current_stream(pred.device)
    rc = lib.fcm_confusion(ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(truth.data_ptr()), pred.numel(),
                           int(n_pred), int(n_truth), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream))
    if rc != L.FCM_OK:
        raise FcmError(rc, "fcm_confusion")
    return out


def dice(counts, n_pred: int, n_truth: int, class_of=None, stream=None):
    """Dice coefficient per ground-truth class (Eq.5) from confusion counts;
    cluster j counts as class class_of[j] (-1: none; None: class j).  Returns
    a float64 device tensor [n_truth] (NaN where both sets are empty)."""
    import torch
    lib = L.load()
    out = torch.empty(int(n_truth), dtype=torch.float64, device=counts.device)
    st = stream if stream is not None else torch.cuda.current_stream(counts.device)
    cls = None
    if class_of is not None:
        arr = (ctypes.c_int32 * int(n_pred))(*[int(v) for v in class_of])
        cls = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
    rc = lib.fcm_dice(ctypes.c_void_p(counts.data_ptr()), int(n_pred), int(n_truth), cls,
                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream))
    if rc != L.FCM_OK:
        raise FcmError(rc, "fcm_dice")
    return out


def rank_classes(centroids, n_truth: int):
    """Cluster -> class map by intensity order: the cluster with the k-th
    smallest centroid is class k (ties by index; ranks >= n_truth map to -1).
    For ground truths whose classes are numbered by increasing mean grey
    level, like the phantom's background, CSF, GM, WM."""
    order = sorted(range(len(centroids)), key=lambda j: (float(centroids[j]), j))
    cls = [-1] * len(centroids)
    for r, j in enumerate(order):
        cls[j] = r if r < n_truth else -1
    return cls


class MLP:
    """Histogram -> centroid network (256 -> 128 -> 64 -> C), trained and run
    by the library's kernels.  Inputs are normalised histograms (float32
    device tensors [B, 256]); outputs and targets are centroids / 255."""

    def __init__(self, n_clusters: int, seed: int = 0, stream=None):
        import torch
        self._lib = L.load()
        self.C = int(n_clusters)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = ctypes.c_void_p()
        rc = self._lib.fcm_mlp_create(ctypes.byref(self._h), self.C, ctypes.c_uint64(seed),
                                      ctypes.c_void_p(self._stream.cuda_stream))
        if rc != L.FCM_OK:
            self._h = None
            raise FcmError(rc, "fcm_mlp_create")
        self.n_params = int(self._lib.fcm_mlp_param_count(self.C))

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(self._lib.fcm_mlp_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    "fcm_mlp_get_params")
        return out

    def set_params(self, theta):
        buf = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
        if buf.shape != (self.n_params,):
            raise ValueError(f"expected {self.n_params} parameters")
        self._check(self._lib.fcm_mlp_set_params(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    "fcm_mlp_set_params")

    def forward(self, hist, bf16: bool = False):
        import torch
        hist = self._dev2d(hist, 256)
        out = torch.empty((hist.shape[0], self.C), dtype=torch.float32, device=hist.device)
        self._check(self._lib.fcm_mlp_forward(self._h, ctypes.c_void_p(hist.data_ptr()), hist.shape[0],
                                              ctypes.c_void_p(out.data_ptr()),
                                              L.FCM_MLP_BF16 if bf16 else L.FCM_MLP_FP32), "fcm_mlp_forward")
        return out

    def loss_grad(self, hist, target):
        hist, target = self._dev2d(hist, 256), self._dev2d(target, self.C)
        loss = ctypes.c_double()
        g = np.empty(self.n_params, dtype=np.float32)
        self._check(self._lib.fcm_mlp_loss_grad(self._h, ctypes.c_void_p(hist.data_ptr()),
                                                ctypes.c_void_p(target.data_ptr()), hist.shape[0],
                                                ctypes.byref(loss), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    "fcm_mlp_loss_grad")
        return loss.value, g

    def train(self, hist, target, epochs: int, batch: int = 256, lr: float = 1e-3, seed: int = 0):
        hist, target = self._dev2d(hist, 256), self._dev2d(target, self.C)
        cfg = L.FcmTrainCfg(epochs=int(epochs), batch=int(batch), lr=float(lr), pad=0, seed=int(seed))
        losses = np.empty(int(epochs), dtype=np.float64)
        self._check(self._lib.fcm_mlp_train(self._h, ctypes.c_void_p(hist.data_ptr()),
                                            ctypes.c_void_p(target.data_ptr()), hist.shape[0], ctypes.byref(cfg),
                                            losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "fcm_mlp_train")
        return losses

    def warm_centroids(self, hist):
        """Start centroids [B, C] (float64 device tensor; NaN rows = no valid start)."""
        import torch
        hist = self._dev2d(hist, 256)
        out = torch.empty((hist.shape[0], self.C), dtype=torch.float64, device=hist.device)
        self._check(self._lib.fcm_warm_centroids(self._h, ctypes.c_void_p(hist.data_ptr()), hist.shape[0],
                                                 ctypes.c_void_p(out.data_ptr()),
                                                 ctypes.c_void_p(self._stream.cuda_stream)), "fcm_warm_centroids")
        return out

    def save(self, path: str):
        """Write the parameters to a network file (fcm_mlp_save)."""
        self._check(self._lib.fcm_mlp_save(self._h, os.fsencode(path)), "fcm_mlp_save")

    def load(self, path: str):
        """Read parameters written by save() into this network (fcm_mlp_load)."""
        self._check(self._lib.fcm_mlp_load(self._h, os.fsencode(path)), "fcm_mlp_load")

    @staticmethod
    def _dev2d(t, cols):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
            raise TypeError("expected a float32 CUDA/HIP tensor")
        t = t.contiguous()
        if t.dim() != 2 or t.shape[1] != cols or t.shape[0] < 1:
            raise ValueError(f"expected shape [B, {cols}]")
        return t

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fcm_mlp_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # at interpreter shutdown the HIP runtime (and any profiler attached
        # to it) may already be torn down: release nothing then
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if self._h is None:
            raise FcmError(L.FCM_ESTATE, what)
        if rc != L.FCM_OK:
            raise FcmError(rc, what)
