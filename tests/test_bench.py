"""Host-side checks of bench.py's contract: the one-GPU guard, the algorithmic FLOP count
behind roofline.achieved, and that stored counter traffic is only reported for the
kernel source and workload it was measured on."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_flop_per_eval_tower4():
    # 42 spheres, 40 boxes, 4 blocks, 32 waypoints per segment: the per-evaluation count
    # the roofline of the bench workload is computed from
    assert bench.flop_per_eval(42, 40, 4, 32) == pytest.approx(20983.9375)
    # every term grows with the scene: more boxes, spheres or blocks cost more
    base = bench.flop_per_eval(42, 40, 4, 32)
    assert bench.flop_per_eval(42, 41, 4, 32) > base
    assert bench.flop_per_eval(43, 40, 4, 32) > base
    assert bench.flop_per_eval(42, 40, 5, 32) > base


def _summary_fields(workload):
    fields = {}
    for line in open(os.path.join(ROOT, "profiles", f"k_traj_{workload}_counters.md")):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    return fields


def _source_hash():
    h = hashlib.sha256()
    for name in (("csrc", "kernels.hip"), ("build.py",)):
        with open(os.path.join(ROOT, "paper_2510_07674_amd", *name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def test_stored_traffic_is_gated():
    """Counter figures are reported only for the workload they were taken on, and only
    while the kernel source and build flags hash to the recorded value."""
    for other in ("tiny", "p2p"):
        assert bench.stored_traffic(other) is None and bench.stored_executed_flop(other) is None
    sha = _source_hash()
    for workload in ("tower4", "tower10"):
        fields = _summary_fields(workload)
        assert fields["workload"] == workload
        got, flop = bench.stored_traffic(workload), bench.stored_executed_flop(workload)
        if sha == fields["kernels_sha256"]:
            assert got == float(fields["traffic_bytes_per_launch"])
            assert flop == float(fields["executed_fp32_flop_per_launch"])
        else:
            assert got is None and flop is None
