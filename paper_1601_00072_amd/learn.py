"""Learned warm start: training targets from the GPU solver, training, and
the evaluation against the evenly spaced start.

Targets are the centroids that the batched GPU FCM (Algorithm 1 from the
evenly spaced start) converges to, sorted and divided by 255; inputs are the
instances' normalised histograms, computed on the GPU.  The network is
trained by the library's kernels (fcm_mlp_train) and proposes start
centroids through BF16 inference; Algorithm 1 then runs from them unchanged.
The plain start stays the reference: a warm result is kept only if its J_m is
within 1e-6 (relative) of the plain one.
"""
from __future__ import annotations

import time

import numpy as np

from .api import FCM, MLP, FCMBatch, histogram

J_REL = 1e-6


def upload(instances, device):
    """Concatenate uint8 arrays into one device tensor; returns (tensor, sizes)."""
    import torch
    sizes = [int(a.size) for a in instances]
    flat = np.concatenate([np.ascontiguousarray(a, dtype=np.uint8).ravel() for a in instances])
    return torch.from_numpy(flat).to(device), sizes


def targets(x, sizes, C: int = 4, m: float = 2.0, eps: float = 1e-5, max_iter: int = 300, chunk: int = 4096):
    """GPU-converged centroids / 255 (sorted) of every instance, float32
    device tensor [count, C] (fcm_batch_targets), and the results (in chunks
    of `chunk` instances per batched launch)."""
    import torch
    res = []
    out = torch.empty((len(sizes), C), dtype=torch.float32, device=x.device)
    off = np.concatenate([[0], np.cumsum(sizes)])
    for c0 in range(0, len(sizes), chunk):
        c1 = min(len(sizes), c0 + chunk)
        sub = x[int(off[c0]):int(off[c1])]
        with FCMBatch(sub, sizes[c0:c1], [dict(n_clusters=C, m=m, eps=eps, max_iter=max_iter)] * (c1 - c0)) as b:
            res.extend(b.solve())
            b.targets(C, out[c0:c1])
    return out, res


def train(x, sizes, C: int = 4, epochs: int = 60, batch: int = 256, lr: float = 1e-3, seed: int = 1,
          m: float = 2.0):
    """Train a network on the instances in x.  Returns (net, epoch losses,
    seconds for targets, seconds for training)."""
    import torch
    t0 = time.perf_counter()
    hist = histogram(x, sizes)
    tgt, _ = targets(x, sizes, C=C, m=m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net = MLP(C, seed=seed)
    losses = net.train(hist, tgt, epochs=epochs, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return net, losses, t1 - t0, t2 - t1


def evaluate_instances(net, x, sizes, C: int = 4, m: float = 2.0, eps: float = 1e-5, reps: int = 1):
    """Per instance, one handle each: plain solve (evenly spaced start) and
    warm solve with the fall-back check, then timed re-runs of both (plain:
    reset + solve; warm: histogram + network + solve, no check).  Returns a
    dict of per-instance arrays and summary figures."""
    import torch
    off = np.concatenate([[0], np.cumsum(sizes)])
    it_p, it_w, used, jrel, t_p, t_w = [], [], [], [], [], []
    for i in range(len(sizes)):
        xi = x[int(off[i]):int(off[i + 1])]
        with FCM(xi, C, m=m, eps=eps) as f:
            rw, u, rp = f.solve_warm(net, check=True)
            it_p.append(rp.iters)
            it_w.append(rw.iters)
            used.append(u)
            jrel.append((rw.J - rp.J) / rp.J if rp.J > 0 else 0.0)
            torch.cuda.synchronize()
            s = time.perf_counter()
            for _ in range(reps):
                f.reset()
                f.solve()
            torch.cuda.synchronize()
            t_p.append((time.perf_counter() - s) / reps)
            s = time.perf_counter()
            for _ in range(reps):
                f.solve_warm(net, check=False)
            torch.cuda.synchronize()
            t_w.append((time.perf_counter() - s) / reps)
    it_p, it_w, used = np.array(it_p), np.array(it_w), np.array(used)
    jrel = np.array(jrel)
    it_eff = np.where(used, it_w, it_p)
    t_p, t_w = np.array(t_p), np.array(t_w)
    return {
        "instances": len(sizes),
        "iters_plain_mean": float(it_p.mean()), "iters_warm_mean": float(it_eff.mean()),
        "iters_plain_median": float(np.median(it_p)), "iters_warm_median": float(np.median(it_eff)),
        "fallback_rate": float(1.0 - used.mean()),
        # (J_warm - J_plain) / J_plain over the accepted warm results: at most
        # 1e-6 by the rule; a clearly negative gap is a lower minimum found
        "max_rel_J_excess_accepted": float(np.max(jrel[used])) if used.any() else 0.0,
        "lower_minimum_count": int(np.count_nonzero(used & (jrel < -1e-6))),
        "same_minimum_max_rel_J_gap": float(np.max(np.abs(jrel[used & (jrel >= -1e-6)]), initial=0.0)),
        "ms_plain_mean": float(t_p.mean() * 1e3), "ms_warm_mean": float(t_w.mean() * 1e3),
        "time_ratio_warm_over_plain": float(t_w.sum() / t_p.sum()),
    }


def evaluate_batch(net, x, sizes, C: int = 4, m: float = 2.0, eps: float = 1e-5, reps: int = 3):
    """All instances in one batched launch: plain vs warm (histograms +
    network + solve) wall time, and the per-instance iterations with the
    fall-back check."""
    import torch
    params = [dict(n_clusters=C, m=m, eps=eps)] * len(sizes)
    with FCMBatch(x, sizes, params) as b:
        warm, used, plain = b.solve_warm(net, check=True)
        b.set_start(None)
        b.solve()
        torch.cuda.synchronize()
        s = time.perf_counter()
        for _ in range(reps):
            b.set_start(None)
            b.solve()
        torch.cuda.synchronize()
        tp = (time.perf_counter() - s) / reps
        s = time.perf_counter()
        for _ in range(reps):
            b.set_start(net)
            b.solve()
        torch.cuda.synchronize()
        tw = (time.perf_counter() - s) / reps
    ip = np.array([r.iters for r in plain])
    iw = np.array([r.iters for r in warm])
    return {
        "instances": len(sizes), "ms_plain": tp * 1e3, "ms_warm": tw * 1e3, "time_ratio_warm_over_plain": tw / tp,
        "iters_plain_mean": float(ip.mean()), "iters_warm_mean": float(iw.mean()),
        "iters_plain_max": int(ip.max()), "iters_warm_max": int(iw.max()),
        "fallback_rate": float(1.0 - np.mean(used)),
    }
