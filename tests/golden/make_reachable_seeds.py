"""Writes reachable_seeds.txt: the point-to-point scene seeds (workload p2p) whose start
and goal configurations penetrate no box (zero clutter score: no robot sphere inside an
obstacle), certified with the FP64 oracle (test infrastructure).  The tower and
fixed-goal workloads are built around a known plan instead (make_witness_scenes.py).

    python tests/golden/make_reachable_seeds.py [--count 32]
"""
import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2510_07674_amd import synth  # noqa: E402

WORKLOADS = ("p2p",)


def certify(name, seed):
    prob, pr, _ = synth.config(name, seed)
    o = oracle.Oracle(prob, pr)
    pose = np.zeros((prob.B, 4))
    return o.arm_clutter(prob.q_home, pose, 0, 2) == 0.0 and o.arm_clutter(prob.p2p_goal, pose, 0, 2) == 0.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=32, help="certified seeds to list")
    args = ap.parse_args()
    oracle.build(force=False)
    path = os.path.join(HERE, "reachable_seeds.txt")
    lines = []
    for name in WORKLOADS:
        seeds, s = [], 0
        while len(seeds) < args.count:
            if certify(name, s):
                seeds.append(s)
            s += 1
        lines.append(f"{name} " + " ".join(map(str, seeds)))
        print(f"{name}: {len(seeds)} of the first {s} seeds certified", flush=True)
    with open(path, "w") as f:
        f.write("# point-to-point scene seeds with collision-free ends, certified by make_reachable_seeds.py (oracle)\n")
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
