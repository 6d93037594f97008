"""Benchmark of the FCM hot path on one MI355X.

A step is one whole solve on a resident input: the data-range pass and v^0,
fused passes until max |dU| < eps, and the defuzzified labels.  Headline
workload: the largest single-GPU volume, the 512x512x256 (67,108,864-voxel)
ellipsoid-shell phantom, seed 3, noise sigma 9, bias 20 %, C = 4, m = 2,
eps = 1e-5, max 300 iterations.

Prints one JSON line.  ``value`` = voxel-iterations/s = n * passes / wall time
of the timed steps (passes = T + 1 per solve, counted on the device).
``roofline`` refers to the dominant kernel, the persistent solve kernel (one
launch per solve runs the data-range pass and every fused pass): achieved
voxel-passes per second of launch time (HIP events on the solve's stream)
against the ALU roofline of a fixed count of lane-ops per voxel-iteration
(``fixed_ops``), with the library's own op count beside it.
``cpu_baseline`` is the FP64 oracle timed on the host on the same volume.
``extra`` holds the other measured workloads (the 128x128x64 volume, the
200x200 slice and the per-pass latency floor, the 512-instance batch, the
learned warm start, the histogram-domain driver, Dice, the paper's protocol
and the paper's GPU design); ``--quick`` skips them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.  Rates of the fixed count:
# packed FP32 add/mul/fma 7.86e13 lane-op/s (157.3 TFLOP/s / 2), unpacked ops
# (max, compare) 3.93e13, transcendentals (rcp, sqrt, exp2, log2) at quarter
# rate 9.83e12.
RATE_PACKED = 256 * 4 * 16 * 2.4e9 * 2
RATE_UNPACKED = 256 * 4 * 16 * 2.4e9
RATE_TRANS = RATE_UNPACKED / 4
PEAK_LANE_OPS = RATE_UNPACKED  # one FP32 VALU op per lane per cycle (this build: no packed FP32)
HBM_PEAK = 8.0e12
METRIC = "FCM voxel-iterations/s & time-to-converge (eps=1e-5) vs plain init, % roofline"


def fixed_ops(C: int, m: float):
    """Lane-ops per voxel-iteration fixed in advance from the method (not from
    the kernel): (packable add/mul/fma, unpacked, transcendental).
    One membership evaluation (Eq.4): m = 2: 4C - 1 add/mul and C + 1
    transcendentals; m = 1.5: 5C - 1 and C + 1; other m: 5C - 1 and 2C + 1.
    A pass evaluates the new and the previous memberships (two evaluations),
    then u^m (m = 2: C mul; 1.5: C sqrt + C mul; other: C sqrt + 2C mul),
    the Eq.3/Eq.1 accumulations (3C) and the change test (C sub, C max)."""
    if m == 2.0:
        ev, tr, um, umt = 4 * C - 1, C + 1, C, 0
    elif m == 1.5:
        ev, tr, um, umt = 5 * C - 1, C + 1, C, C
    else:
        ev, tr, um, umt = 5 * C - 1, 2 * C + 1, 2 * C, C
    return 2 * ev + um + 3 * C + C, C, 2 * tr + umt


def alu_ceiling(C: int, m: float) -> float:
    """Voxel-iterations/s at the ALU roofline of the fixed count (each class
    at its own rate, one shared issue)."""
    p, u, t = fixed_ops(C, m)
    return 1.0 / (p / RATE_PACKED + u / RATE_UNPACKED + t / RATE_TRANS)


def alg_lane_ops(C: int, m: float, with_old: bool = True) -> float:
    """The library's own count of VALU lane-op slots per voxel for one fused
    pass (the membership forms it uses; reported beside the fixed count).

    Counts the arithmetic of Eq.1, Eq.3, Eq.4 and the stopping test with the
    fused forms the ISA offers (fma where a product feeds a sum, max3 for
    running maxima) and transcendentals weighted 4.  Excludes byte-to-float
    conversion, Kahan compensation, range/separation tests and all reductions.
      m = 2, one evaluation (product form):
        C sub + C mul (q) + (3C - 6) mul (leave-one-out products)
        + (C - 1) add (sum) + 4 (rcp) + C mul (scale)          = 7C - 3
      m other, one evaluation (m = 2 form, then u2^alpha normalised):
        7C - 3 + 4C (log2) + C/2 (max3) + C mul + 4C (exp2) + (C - 1) add
        + 4 (rcp) + C mul                                      = 18.5C + 0
      change test: C sub + C/2 (max3)
      weights, sums, objective:
        m = 2: C mul (u^2) + C fma (num) + C add (den) + 1 fma (J)
        other: 4 (log2 S) + C fma + 4C (exp2) + C fma + C add + C fma (J)
    """
    if m == 2.0:
        ev = 7 * C - 3
        tail = 3 * C + 1
    else:
        ev = 18.5 * C
        tail = 4 + 8 * C
    ops = ev + tail
    if with_old:
        ops += ev + 1.5 * C
    return float(ops)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--shape", default="256,512,512", help="D,H,W (or H,W) of the phantom")
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--sigma", type=float, default=9.0, help="noise sigma of the phantom")
    ap.add_argument("--bias", type=float, default=0.2, help="bias-field amplitude of the phantom")
    ap.add_argument("--clusters", type=int, default=4)
    ap.add_argument("--m", type=float, default=2.0)
    ap.add_argument("--eps", type=float, default=1e-5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--extras", default="all",
                    help="comma-separated extras to run (small,batched,learned,histogram,quality,protocol,design)")
    ap.add_argument("--launch", choices=("cooperative", "resident"), default="resident",
                    help="launch of the persistent solve kernel")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuner cache file (a matching entry is applied without timing)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device 5 times (counter calibration)")
    return ap.parse_args()


def cpu_baseline(x_np, C, m, eps, budget_s):
    """The oracle on the same volume.  Oracle-F (plain C, FP64, one static
    chunk of voxels per thread) on the host's cores -- at most 16, the CPU
    share of one GPU -- runs the whole solve over every voxel; the literal
    numpy oracle on one core runs on a bounded sample (at most 2^20 voxels
    from the middle of the volume) until converged or until the time budget
    is spent.  Both in voxel-iterations/s; the threaded figure is the
    baseline."""
    import numpy as np

    from oracle import fcm_fast, fcm_ref
    x = x_np.ravel()
    n = x.size
    host = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = host
    threads = max(1, min(16, avail))
    fcm_fast.solve(x[:4096], C, m=m, eps=eps, threads=threads)  # load the library
    t0 = time.perf_counter()
    tr = fcm_fast.solve(x, C, m=m, eps=eps, max_iter=300, threads=threads)
    el_f = time.perf_counter() - t0
    passes_f = tr.T + 1
    # literal oracle, one core, on a bounded sample of the same volume
    ns = min(n, 1 << 20)
    s0 = (n - ns) // 2
    xs = x[s0:s0 + ns]
    t0 = time.perf_counter()
    v = fcm_ref.linspace_init(int(xs.min()), int(xs.max()), C)
    U = fcm_ref.memberships(xs, v, m)
    passes = 1
    t = 0
    while True:
        t += 1
        v = fcm_ref.centroids(xs, U, m, v)
        U_new = fcm_ref.memberships(xs, v, m)
        delta = float(np.max(np.abs(U_new - U)))
        U = U_new
        passes += 1
        if delta < eps or time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": n * passes_f / el_f, "unit": "voxel-iterations/s", "cores": threads, "kind": "oracle",
            "host_cpu_count": host, "cpus_available": avail,
            "sample": f"the whole solve ({tr.T} iterations, {passes_f} membership sweeps) of the FP64 C oracle "
                      f"(Oracle-F, per voxel, {threads} threads of {avail} available, {host} on the host) over all "
                      f"{n} voxels of the same volume: {el_f:.3f} s",
            "literal_single_core": {"value": ns * passes / el, "unit": "voxel-iterations/s", "cores": 1,
                                    "sample": f"{t} iterations ({passes} membership evaluations) of the FP64 "
                                              f"literal numpy oracle over voxels {s0}..{s0 + ns - 1} of the same "
                                              f"volume: {el:.2f} s"}}


def timed_solves(f, steps, labels=None):
    """Run `steps` solves (reset + solve [+ labels]); returns (seconds, passes, kernel_ms, last result)."""
    import torch
    passes, kms, r = 0, 0.0, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f.reset()
        r = f.solve()
        if labels is not None:
            f.labels(labels)
        passes += r.passes
        kms += r.kernel_ms
    torch.cuda.synchronize()
    return time.perf_counter() - t0, passes, kms, r


def timed_async(f, steps, labels):
    """`steps` whole solves, each with its labels, enqueued back to back
    (fcm_solve_async: one persistent launch per solve that also writes the
    labels, no host wait), then one wait.  Returns (seconds, fused passes counted on the device, summed launch
    time in ms, last result)."""
    import torch
    _, tot0 = f.result()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        f.solve_async(labels)
    r, tot = f.result()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, tot - tot0, r.kernel_ms, r


PROFILES = os.path.join(ROOT, "profiles")
TUNE_CACHE = os.path.join(ROOT, "paper_1601_00072_amd", "tuning_mi355x.txt")


def kernel_sources(C: int) -> list:
    """The files the persistent kernel for C clusters is compiled from: its
    translation unit and every quoted include it reaches, recursively."""
    import re
    dirs = [os.path.join(ROOT, "paper_1601_00072_amd", "csrc"), os.path.join(ROOT, "include")]
    todo, seen = [os.path.join(dirs[0], f"fcm_pass_c{C}.hip")], []
    while todo:
        path = todo.pop()
        if path in seen:
            continue
        seen.append(path)
        with open(path) as fh:
            for inc in re.findall(r'^\s*#\s*include\s+"([^"]+)"', fh.read(), flags=re.M):
                for d in dirs:
                    cand = os.path.join(d, inc)
                    if os.path.exists(cand):
                        todo.append(cand)
                        break
    return sorted(seen)


def sources_digest(C: int = 4) -> str:
    """SHA-256 prefix over the sources of the persistent kernel (kernel_sources)."""
    import hashlib
    h = hashlib.sha256()
    for path in kernel_sources(C):
        h.update(os.path.relpath(path, ROOT).encode())
        h.update(b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def tuning_tag(t) -> str:
    return f"grid={t['grid']},unroll={t['unroll']},exchange={t['exchange']},launch={t['launch']}"


def recorded(key, shape, C, m, tuning):
    """A machine-readable line `key: value ... sources_digest: D tuning: T
    workload: W C=.. m=..` from the committed profile summaries, as a dict of
    its fields, or None when none was taken on the current kernel sources,
    this workload and this launch configuration."""
    import glob
    for path in sorted(glob.glob(os.path.join(PROFILES, "*.md"))):
        try:
            with open(path) as fh:
                lines = fh.readlines()
        except OSError:
            continue
        for line in lines:
            f = line.split()
            if f[:1] != [key + ":"]:
                continue
            kv = dict(zip(f[0::2], f[1::2]))
            if (kv.get("sources_digest:") == sources_digest(C) and kv.get("tuning:") == tuning_tag(tuning)
                    and kv.get("workload:") == ",".join(map(str, shape)) and f"C={C}" in f and f"m={float(m)}" in f):
                return {k.rstrip(":"): v for k, v in kv.items()}
    return None


def recorded_traffic(shape, C, m, tuning):
    """HBM bytes per launch of the persistent kernel (copy-calibrated
    FETCH_SIZE + WRITE_SIZE) from the committed summaries, or None."""
    kv = recorded("traffic_bytes_per_launch", shape, C, m, tuning)
    return None if kv is None else int(kv["traffic_bytes_per_launch"])


def recorded_counters(shape, C, m, tuning):
    """VALU counters of the persistent kernel per voxel-pass from the
    committed summaries (rocprofv3 --pmc), or None."""
    kv = recorded("valu_counters", shape, C, m, tuning)
    if kv is None:
        return None
    out = {}
    for k, v in kv.items():
        if k in ("valu_counters", "sources_digest", "tuning", "workload") or "=" in k:
            continue
        try:
            out[k] = float(v)
        except ValueError:
            out[k] = v
    return out


def roofline(n, C, m, passes_per_launch, launch_s):
    """Achieved rates of one launch: voxel-passes per second, and the
    library's own lane-op count per second (the first pass evaluates one
    membership set, the others two)."""
    vox = n * passes_per_launch / launch_s
    ops = n * (alg_lane_ops(C, m, False) + (passes_per_launch - 1) * alg_lane_ops(C, m, True))
    return vox, ops / launch_s


def roofline_entry(shape, n, C, m, passes_per_launch, launch_s, tuning, kernel):
    vox, ops = roofline(n, C, m, passes_per_launch, launch_s)
    ceil = alu_ceiling(C, m)
    p, u, t = fixed_ops(C, m)
    return {
        "bound": "alu",
        "kernel": kernel,
        "achieved": vox,
        "peak": ceil,
        "unit": "voxel-iterations/s",
        "frac": vox / ceil,
        "traffic": recorded_traffic(shape, C, m, tuning),
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "launch_avg_us": launch_s * 1e6,
        "passes_per_launch": passes_per_launch,
        "peak_basis": f"fixed count per voxel-iteration: {p} packable add/mul/fma, {u} unpacked, {t} "
                      f"transcendental lane-ops at {RATE_PACKED:.3g} / {RATE_UNPACKED:.3g} / {RATE_TRANS:.3g} "
                      f"per s (256 CUs x 4 SIMD x 16 lanes, 2.4 GHz)",
        "library_count": {"lane_ops_per_voxel_pass": alg_lane_ops(C, m, True), "achieved_T_lane_op_s": ops / 1e12,
                          "peak_T_lane_op_s": PEAK_LANE_OPS / 1e12, "frac": ops / PEAK_LANE_OPS},
        "hbm": {"algorithmic_GB_s": vox / 1e9, "frac_of_8TB_s": vox / HBM_PEAK},
        "counters": recorded_counters(shape, C, m, tuning),
    }


def solve_steps(dev, x, C, m, eps, steps, warmup, launch, autotune, tune_cache):
    """The timed steps on one resident input: `warmup` + `steps` whole solves
    with labels enqueued back to back (fcm_solve_async), then the same solves
    waited for one at a time (fcm_solve + fcm_labels)."""
    import torch

    from paper_1601_00072_amd import FCM
    labels = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)
    f = FCM(x, C, m=m, eps=eps, max_iter=300, timing=True, stream=stream)
    f.set_tuning(launch=0 if launch == "cooperative" else 1)
    if autotune:
        f.autotune(cache=tune_cache, reps=3)
    timed_async(f, warmup, labels)
    tuning = f.tuning
    el, passes_total, kernel_ms_total, r = timed_async(f, steps, labels)
    el_sync, passes_sync, _, _ = timed_solves(f, steps, labels)
    f.close()
    return {"el": el, "passes": passes_total, "kernel_ms": kernel_ms_total, "r": r, "tuning": tuning,
            "el_sync": el_sync, "passes_sync": passes_sync, "steps": steps}


def small_workloads(dev, steps, launch, tune_cache):
    """Configs small enough that a pass is latency-bound: the 200x200 slice
    (the paper's 40 KB point) and the 128x128x64 volume (its ~1 MB point):
    time to converge, voxel-iterations/s, time per pass against the ALU time
    of a pass at the roofline; the slice's time per pass is the per-pass
    latency floor of the persistent solve."""
    import torch

    from phantom import PhantomParams, phantom
    out = {}
    cases = (("slice_200x200", (200, 200), 1, "0.08 s at 40 KB (Table 3, Tesla C2050), context only"),
             ("volume_128x128x64", (64, 128, 128), 2, "2.33 s at 1 MB (Table 3, Tesla C2050), context only"))
    for name, shape, seed, ctx in cases:
        x = torch.from_numpy(phantom(PhantomParams(shape=shape, seed=seed)).ravel()).to(dev)
        n = x.numel()
        st = solve_steps(dev, x, 4, 2.0, 1e-5, steps, 5, launch, True, tune_cache)
        r = st["r"]
        pps = st["passes"] / steps
        launch_s = st["kernel_ms"] / steps * 1e-3
        ent = roofline_entry(shape, n, 4, 2.0, pps, launch_s, st["tuning"], "fcm_persist_kernel<4>")
        out[name] = {
            "workload": f"ellipsoid-shell phantom {'x'.join(map(str, shape[::-1]))} ({n} voxels), seed {seed}, "
                        f"sigma 8, bias 10%, C=4, m=2, eps=1e-5",
            "iterations": r.iters, "passes_per_solve": pps,
            "time_to_converge_ms": st["el"] * 1e3 / steps,
            "time_to_converge_ms_host_waits_each_solve": st["el_sync"] * 1e3 / steps,
            "voxel_iterations_per_s": n * st["passes"] / st["el"],
            "us_per_pass": launch_s / pps * 1e6,
            "alu_us_per_pass_at_roofline": n / alu_ceiling(4, 2.0) * 1e6,
            "roofline": ent, "tuning": st["tuning"], "paper_context": ctx,
        }
    out["latency_floor_us_per_pass"] = out["slice_200x200"]["us_per_pass"]
    return out


def histogram_domain(dev, cases):
    """Exact histogram-domain solve (FCM_DRIVER_HISTOGRAM) on the given
    volumes ((name, device tensor) pairs): one pass over the data, then the
    iteration over grey levels; time to converge with labels, against the
    per-voxel persistent solve on the same handle configuration."""
    import torch

    from paper_1601_00072_amd import FCM
    out = {}
    for name, x in cases:
        labels = torch.empty_like(x)
        res = {}
        for drv in (3, 2):
            with FCM(x, 4) as f:
                f.set_tuning(driver=drv)
                timed_solves(f, 2, labels)
                el, passes, _, r = timed_solves(f, 10, labels)
            res[drv] = (el / 10 * 1e3, r.iters)
        out[name] = {"ms_to_converge_histogram": res[3][0], "iterations_histogram": res[3][1],
                     "ms_to_converge_per_voxel": res[2][0], "iterations_per_voxel": res[2][1],
                     "speedup": res[2][0] / res[3][0]}
    return out


def paper_protocol(dev, x, shape):
    """The paper's own protocol on the given volume (the 128x128x64 one): random memberships U^0
    (five seeds), centroids first, eps = 0.005; iterations, time to converge
    (labels included) and the final centroids, beside the evenly spaced
    start at the same eps."""
    import torch

    from paper_1601_00072_amd import FCM
    labels = torch.empty_like(x)
    runs = []
    for seed in range(1, 6):
        with FCM(x, 4, eps=0.005, init=("random_u", seed)) as f:
            timed_solves(f, 2, labels)
            el, _, _, r = timed_solves(f, 10, labels)
        runs.append({"seed": seed, "iterations": r.iters, "ms_to_converge": el / 10 * 1e3,
                     "centroids": [round(float(v), 4) for v in r.centroids]})
    with FCM(x, 4, eps=0.005) as f:
        timed_solves(f, 2, labels)
        el, _, _, r = timed_solves(f, 10, labels)
    return {"workload": "volume " + "x".join(map(str, shape[::-1])) + ", C=4, m=2, eps=0.005",
            "random_u": runs,
            "linspace": {"iterations": r.iters, "ms_to_converge": el / 10 * 1e3,
                         "centroids": [round(float(v), 4) for v in r.centroids]}}


def paper_design(dev, x, shape, fused_ms, eps):
    """The paper's GPU structure (per-cluster kernels, Algorithm 2 reductions,
    U copied to the host every iteration for the stopping test) on the
    given volume (the 128x128x64 one), against the fused persistent solve of the same start."""
    import torch

    from paper_1601_00072_amd import paper_baseline
    out = {}
    for name, init, e in (("linspace start, eps=%g" % eps, None, eps), ("random U^0 seed 3, eps=0.005", ("random_u", 3), 0.005)):
        paper_baseline(x, 4, eps=e, init=init)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            res, _, _, st = paper_baseline(x, 4, eps=e, init=init)
        ms = (time.perf_counter() - t0) / reps * 1e3
        out[name] = {"iterations": res.iters, "ms_per_solve": ms, "loop_ms": st["total_ms"],
                     "kernels_ms": st["kernels_ms"], "copy_ms": st["copy_ms"], "host_test_ms": st["host_ms"],
                     "launches": st["launches"]}
    out["fused_persistent_ms_same_start"] = fused_ms
    out["speedup_fused_vs_paper_design"] = out["linspace start, eps=%g" % eps]["ms_per_solve"] / fused_ms
    return out


def quality(dev, cases):
    """Dice coefficient per tissue (Eq.5) of the GPU segmentations of the
    given phantoms ((name, PhantomParams) pairs) against their tissue labels,
    and the time of the confusion-count + Dice kernels."""
    import torch

    from paper_1601_00072_amd import FCM, confusion, dice, rank_classes
    from phantom import phantom
    out = {}
    for name, p in cases:
        img, lab = phantom(p, with_labels=True)
        x = torch.from_numpy(img.ravel()).to(dev)
        truth = torch.from_numpy(lab.ravel()).to(dev)
        with FCM(x, 4) as f:
            r = f.solve()
            labels = f.labels()
        cls = rank_classes(r.centroids, 4)
        d = dice(confusion(labels, truth, 4, 4), 4, 4, cls)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            d = dice(confusion(labels, truth, 4, 4), 4, 4, cls)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        out[name] = {"dsc": dict(zip(("background", "CSF", "GM", "WM"), d.cpu().tolist())),
                     "us_confusion_and_dice": us, "confusion_GB_per_s": 2 * x.numel() / (us * 1e-6) / 1e9}
        del x, truth, labels
    return out


def batched(dev, tune_cache):
    import numpy as np
    import torch

    from paper_1601_00072_amd import FCM, FCMBatch
    from phantom import batch_instances, phantom
    inst = batch_instances()
    xs = [phantom(p).ravel() for p, _ in inst]
    Cs = [c for _, c in inst]
    flat = torch.from_numpy(np.concatenate(xs)).to(dev)
    n = flat.numel()
    with FCMBatch(flat, [a.size for a in xs], [dict(n_clusters=c, m=2.0, eps=1e-5) for c in Cs]) as b:
        bs, cpt, bgrid, _ = b.autotune(cache=tune_cache, reps=1)
        b.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            res = b.solve()
        torch.cuda.synchronize()
        el_b = (time.perf_counter() - t0) / reps
        tl = [b.timeline(i) for i in range(len(xs))]
    vox_passes = sum(a.size * r.passes for a, r in zip(xs, res))
    # algorithmic work of every instance at its own C and pass count: the
    # fixed count's roofline time, and the library's own lane-op count
    t_roof = sum(a.size * r.passes / alu_ceiling(c, 2.0) for a, c, r in zip(xs, Cs, res))
    ops = sum(a.size * (alg_lane_ops(c, 2.0, False) + (r.passes - 1) * alg_lane_ops(c, 2.0, True))
              for a, c, r in zip(xs, Cs, res))
    # per-instance launch loop: the single-instance solver, one instance after another
    views, off = [], 0
    for a in xs:
        views.append(flat[off:off + a.size])
        off += a.size
    handles = [FCM(v, c) for v, c in zip(views, Cs)]
    for h in handles:
        h.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h in handles:
        h.reset()
        h.solve()
    torch.cuda.synchronize()
    el_l = time.perf_counter() - t0
    for h in handles:
        h.close()
    return {"workload": "512 instances in one persistent launch: 496 slices side U{64..512} + 16 cubes side "
                        "U{96..160}, C_i in 3..8, m=2, eps=1e-5",
            "voxels": n, "max_iterations": max(r.iters for r in res),
            "ms_per_batch_solve": el_b * 1e3, "voxel_iterations_per_s": vox_passes / el_b,
            "ms_per_instance_loop": el_l * 1e3, "speedup_vs_instance_loop": el_l / el_b,
            "roofline_frac_wall": t_roof / el_b,
            "roofline_frac_wall_library_count": ops / el_b / PEAK_LANE_OPS,
            "tiling": {"block": bs, "chunks_per_thread": cpt, "grid": bgrid},
            "timeline": batch_timeline(tl, [a.size for a in xs], t_roof)}


def batch_timeline(tl, sizes, t_roof):
    """What the per-instance commit times of the last batched solve show:
    instances still running and the share of all voxel-passes committed at
    fractions of the launch, and the instance that finished last (its pass
    count and mean pass time).  The roofline line is where a launch that
    kept every lane busy would have committed all the work."""
    import numpy as np
    end = max(float(t[-1]) for t in tl)
    total = sum(s * (len(t) - 1) for s, t in zip(sizes, tl))
    marks = (0.1, 0.25, 0.5, 0.75, 0.9)
    running, done = {}, {}
    for f in marks:
        at = f * end
        running[f"{round(f * 100)}%"] = int(sum(1 for t in tl if t[-1] > at))
        done[f"{round(f * 100)}%"] = float(sum(s * np.count_nonzero(t[1:] <= at) for s, t in zip(sizes, tl)) / total)
    last = max(range(len(tl)), key=lambda i: tl[i][-1])
    t = tl[last]
    return {"launch_us": end, "roofline_us": t_roof * 1e6, "instances_running": running,
            "voxel_passes_committed": done,
            "last_instance": {"voxels": int(sizes[last]), "passes": len(t) - 1,
                              "us_per_pass_mean": float((t[-1] - t[0]) / max(1, len(t) - 1))}}


# ---- learned warm start (training set, held-out slices and volumes) ----------

_SHARED = None  # anonymous shared mapping filled by forked workers


def _fill(job):
    import numpy as np

    from phantom import jittered_params, phantom
    shape, seeds, offs = job
    view = np.frombuffer(_SHARED, dtype=np.uint8)
    n = int(np.prod(shape))
    for sd, o in zip(seeds, offs):
        view[o:o + n] = phantom(jittered_params(shape, sd)).ravel()
    return len(seeds)


def learned_sets(workers: int):
    """The warm start's data: 20,000 training slices 256x256 (seeds 1e6 + i),
    1,024 held-out slices 256x256 (seeds 2e6 + i) and 64 held-out volumes
    128^3 (seeds 3e6 + i), each phantom with its own jittered parameters.
    Generated by forked workers into one shared mapping, before the process
    touches the GPU.  Returns {name: (uint8 array, shape, count)}."""
    import mmap
    import multiprocessing as mp

    import numpy as np
    global _SHARED
    spec = [("train", (256, 256), 20000, 10 ** 6), ("slices", (256, 256), 1024, 2 * 10 ** 6),
            ("volumes", (128, 128, 128), 64, 3 * 10 ** 6)]
    total, base = 0, {}
    for name, shape, count, _ in spec:
        base[name] = total
        total += int(np.prod(shape)) * count
    _SHARED = mmap.mmap(-1, total)
    jobs = []
    for name, shape, count, seed0 in spec:
        n = int(np.prod(shape))
        step = 1 if len(shape) == 3 else 250
        for i0 in range(0, count, step):
            ids = range(i0, min(count, i0 + step))
            jobs.append((shape, [seed0 + i for i in ids], [base[name] + i * n for i in ids]))
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_fill, jobs, chunksize=1)
    buf = np.frombuffer(_SHARED, dtype=np.uint8)
    return {name: (buf[base[name]:base[name] + int(np.prod(shape)) * count], shape, count)
            for name, shape, count, _ in spec}


def learned(dev, sets, volumes, C, m, eps, steps):
    """Train the network on GPU-converged centroids of the training slices,
    then compare warm and plain starts on the held-out sets (one handle per
    instance, and all in one batched launch) and on whole volumes
    ((name, device tensor) pairs)."""
    import numpy as np
    import torch

    from paper_1601_00072_amd import FCM, learn
    out = {}
    arr, shape, count = sets["train"]
    x = torch.from_numpy(np.asarray(arr)).to(dev)
    sizes = [int(np.prod(shape))] * count
    net, losses, t_tgt, t_train = learn.train(x, sizes, C=4, epochs=100, batch=256, lr=1e-3, seed=1)
    out["training"] = {"phantoms": count, "shape": list(shape), "epochs": 100, "batch": 256, "lr": 1e-3,
                       "loss_first_epoch": float(losses[0]), "loss_last_epoch": float(losses[-1]),
                       "s_targets_gpu_fcm": t_tgt, "s_training": t_train}
    del x
    print(f"# learned: trained ({t_train:.2f} s), loss {losses[0]:.3e} -> {losses[-1]:.3e}", file=sys.stderr,
          flush=True)
    for name in ("slices", "volumes"):
        arr, shape, count = sets[name]
        x = torch.from_numpy(np.asarray(arr)).to(dev)
        sizes = [int(np.prod(shape))] * count
        out[name] = {"per_instance": learn.evaluate_instances(net, x, sizes, C=4),
                     "batched": learn.evaluate_batch(net, x, sizes, C=4)}
        print(f"# learned: {name} done", file=sys.stderr, flush=True)
        del x
    # whole volumes: time to converge, plain vs warm start
    for name, xv in volumes:
        with FCM(xv, C, m=m, eps=eps) as f:
            rw, used, rp = f.solve_warm(net, check=True)
            f.solve()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                f.reset()
                f.solve()
            torch.cuda.synchronize()
            tp = (time.perf_counter() - t0) / steps
            t0 = time.perf_counter()
            for _ in range(steps):
                f.solve_warm(net, check=False)
            torch.cuda.synchronize()
            tw = (time.perf_counter() - t0) / steps
        out[name] = {"iters_plain": rp.iters, "iters_warm": rw.iters, "warm_accepted": used,
                     "rel_J_gap": (rw.J - rp.J) / rp.J, "ms_to_converge_plain": tp * 1e3,
                     "ms_to_converge_warm": tw * 1e3,
                     "warm_includes": "histogram + BF16 network + start post-processing + solve"}
    net.close()
    return out


def main():
    args = parse()
    sets = None
    if (not args.quick and not args.copy_probe and args.gpus == 1
            and (args.extras == "all" or "learned" in args.extras.split(","))):
        t0 = time.perf_counter()
        sets = learned_sets(min(16, os.cpu_count() or 1))
        print(f"# learned-start data generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    dev = torch.device("cuda:0")
    if args.copy_probe:
        a = torch.empty(args.copy_probe, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 5}))
        return

    from phantom import PhantomParams, phantom

    shape = tuple(int(s) for s in args.shape.split(","))
    params = PhantomParams(shape=shape, seed=args.seed, sigma=args.sigma, bias=args.bias)
    x_np = phantom(params)
    n = x_np.size
    x = torch.from_numpy(x_np.ravel()).to(dev)
    C, m, eps = args.clusters, args.m, args.eps
    wl = (f"ellipsoid-shell phantom {'x'.join(map(str, shape[::-1]))} ({n} voxels, uint8), seed {args.seed}, "
          f"sigma {args.sigma:g}, bias {100 * args.bias:g}%, C={C}, m={m}, eps={eps}, max_iter=300, linspace init")
    print(f"# headline: {wl}", file=sys.stderr, flush=True)
    st = solve_steps(dev, x, C, m, eps, args.steps, args.warmup, args.launch, not args.no_autotune, args.tune_cache)
    r, tuning, el = st["r"], st["tuning"], st["el"]
    print(f"# timed {args.steps} solves: T={r.iters} status={r.status} tuning {tuning}", file=sys.stderr, flush=True)

    ms_per_step = el * 1e3 / args.steps
    passes_per_solve = st["passes"] / args.steps
    launch_s = st["kernel_ms"] / args.steps * 1e-3
    out = {
        "metric": METRIC,
        "value": n * st["passes"] / el,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": wl,
            "n_voxels": n, "C": C, "m": m, "eps": eps, "iterations": r.iters, "status": r.status,
            "passes_per_solve": passes_per_solve,
            "time_to_converge_ms": ms_per_step,
            "step": "data-range pass + fused passes to convergence + labels, one persistent launch per step "
                    "(fcm_solve_async), steps enqueued back to back, one host wait for the timed run; "
                    "passes counted on the device",
            "ms_per_step_host_waits_each_solve": st["el_sync"] * 1e3 / args.steps,
            "value_host_waits_each_solve": n * st["passes_sync"] / st["el_sync"],
            "launch": args.launch,
            "tuning": tuning,
            "autotuned": not args.no_autotune,
            "precision": "FP32 memberships, Kahan-compensated FP32 partial sums, FP64 cross-block reduction and J",
        },
        "roofline": roofline_entry(shape, n, C, m, passes_per_solve, launch_s, tuning, f"fcm_persist_kernel<{C}>"),
    }
    if not args.quick:
        want = set(args.extras.split(",")) if args.extras != "all" else {
            "small", "batched", "learned", "histogram", "quality", "protocol", "design"}
        ex = {}
        x1 = torch.from_numpy(phantom(PhantomParams(shape=(64, 128, 128), seed=2)).ravel()).to(dev)
        if "small" in want or "design" in want:
            ex["small_workloads"] = sm = small_workloads(dev, args.steps, args.launch, args.tune_cache)
            print(f"# small workloads: floor {sm['latency_floor_us_per_pass']:.2f} us/pass", file=sys.stderr,
                  flush=True)
        if "batched" in want:
            ex["batched"] = bt = batched(dev, args.tune_cache)
            print(f"# batch: {bt['ms_per_batch_solve']:.2f} ms/solve", file=sys.stderr, flush=True)
        if "learned" in want and sets is not None:
            ex["learned_warm_start"] = learned(dev, sets, (("volume_128x128x64", x1), ("volume_512x512x256", x)),
                                               C, m, eps, min(args.steps, 10))
        if "histogram" in want:
            ex["histogram_domain"] = hd = histogram_domain(dev, (("volume_128x128x64", x1), ("volume_512x512x256", x)))
            print(f"# histogram domain: {hd}", file=sys.stderr, flush=True)
        if "quality" in want:
            ex["segmentation_quality"] = q = quality(dev, (("volume_128x128x64", PhantomParams(shape=(64, 128, 128),
                                                                                               seed=2)),
                                                           ("volume_512x512x256", params)))
            print(f"# segmentation quality: {q}", file=sys.stderr, flush=True)
        if "protocol" in want:
            ex["paper_protocol"] = pp = paper_protocol(dev, x1, (64, 128, 128))
            print(f"# paper protocol: {pp}", file=sys.stderr, flush=True)
        if "design" in want:
            ex["paper_design_baseline"] = pd = paper_design(dev, x1, (64, 128, 128),
                                                            sm["volume_128x128x64"]["time_to_converge_ms"], eps)
            print(f"# paper design: {pd}", file=sys.stderr, flush=True)
        out["extra"] = ex
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(x_np, C, m, eps, args.cpu_budget_s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
