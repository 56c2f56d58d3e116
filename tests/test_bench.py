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


def _summary_fields():
    fields = {}
    for line in open(os.path.join(ROOT, "profiles", "k_traj_tower4_counters.md")):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    return fields


def test_stored_traffic_is_gated():
    fields = _summary_fields()
    assert fields["workload"] == "tower4"
    for other in ("tower10", "tiny", "p2p"):
        assert bench.stored_traffic(other) is None
    with open(os.path.join(ROOT, "paper_2510_07674_amd", "csrc", "kernels.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    got = bench.stored_traffic("tower4")
    if sha == fields["kernels_sha256"]:
        assert got == float(fields["traffic_bytes_per_launch"])
    else:
        assert got is None
