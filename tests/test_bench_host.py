"""Host-side parts of the benchmark: the fixed op count and its ceiling, the
batch timeline summary, the lookup of recorded counter lines, and the
one-GPU guard.  No GPU is touched."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_fixed_count_and_ceiling():
    # one Eq.4 evaluation for m = 2: 4C - 1 add/mul, C + 1 transcendentals;
    # two evaluations, u^m (C), Eq.3/Eq.1 sums (3C), change test (C sub, C max)
    assert bench.fixed_ops(4, 2.0) == (50, 4, 10)
    assert bench.fixed_ops(8, 2.0) == (2 * 31 + 8 + 24 + 8, 8, 18)
    # general m: 5C - 1 and 2C + 1 per evaluation, u^m by sqrt and two multiplies
    assert bench.fixed_ops(8, 2.5) == (2 * 39 + 16 + 24 + 8, 8, 2 * 17 + 8)
    c4 = 1.0 / (50 / 7.86432e13 + 4 / 3.93216e13 + 10 / 9.8304e12)
    assert bench.alu_ceiling(4, 2.0) == pytest.approx(c4, rel=1e-12)
    assert bench.alu_ceiling(4, 2.0) == pytest.approx(5.70e11, rel=2e-3)
    assert bench.alu_ceiling(8, 2.5) == pytest.approx(1.65e11, rel=1e-2)
    # the ceiling falls with C and with the general-m form
    assert bench.alu_ceiling(8, 2.0) < bench.alu_ceiling(4, 2.0)
    assert bench.alu_ceiling(4, 2.5) < bench.alu_ceiling(4, 2.0)


def test_batch_timeline_summary():
    # two instances: 100 voxels x 3 passes ending at 13 us, 10 voxels x 10 passes ending at 21 us
    tl = [np.array([1.0, 5.0, 9.0, 13.0]), np.arange(1.0, 22.0, 2.0)]
    s = bench.batch_timeline(tl, [100, 10], 1e-5)
    assert s["launch_us"] == 21.0 and s["roofline_us"] == pytest.approx(10.0)
    assert s["instances_running"] == {"10%": 2, "25%": 2, "50%": 2, "75%": 1, "90%": 1}
    # at 50 % (10.5 us): passes at 5, 9 of the first (200 vox-passes), 3, 5, 7, 9 of the second (40) of 400
    assert s["voxel_passes_committed"]["50%"] == pytest.approx(240 / 400)
    assert s["last_instance"] == {"voxels": 10, "passes": 10, "us_per_pass_mean": 2.0}


def test_recorded_lines(tmp_path, monkeypatch):
    t = dict(grid=512, unroll=2, exchange=3, launch=1)
    dig = bench.sources_digest(4)
    lines = [
        f"    traffic_bytes_per_launch: 1234 sources_digest: {dig} tuning: {bench.tuning_tag(t)} "
        "workload: 256,512,512 C=4 m=2.0",
        f"    valu_counters: v1 valu_insts_per_voxel_pass: 62.9 valu_busy_pct: 91.0 sources_digest: {dig} "
        f"tuning: {bench.tuning_tag(t)} workload: 256,512,512 C=4 m=2.0",
        "    traffic_bytes_per_launch: 999 sources_digest: 0000000000000000 tuning: "
        f"{bench.tuning_tag(t)} workload: 64,128,128 C=4 m=2.0",
    ]
    (tmp_path / "x.md").write_text("\n".join(lines) + "\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.recorded_traffic((256, 512, 512), 4, 2.0, t) == 1234
    assert bench.recorded_counters((256, 512, 512), 4, 2.0, t) == {"valu_insts_per_voxel_pass": 62.9,
                                                                   "valu_busy_pct": 91.0}
    # another workload, launch configuration or source digest: nothing recorded
    assert bench.recorded_traffic((64, 128, 128), 4, 2.0, t) is None
    assert bench.recorded_traffic((256, 512, 512), 4, 2.0, dict(t, grid=256)) is None
    assert bench.recorded_traffic((256, 512, 512), 8, 2.0, t) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--quick"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]
