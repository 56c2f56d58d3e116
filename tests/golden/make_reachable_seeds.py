"""Writes reachable_seeds.txt: for each solve workload, the scene seeds whose problem is
kinematically feasible, certified with the FP64 oracle (test infrastructure):

  * every block's top-down grasp at its initial pose is reached (IK error < 1e-4) from at
    least one of 32 starts drawn uniformly over the joint limits, and
  * for every tower slot height (or fixed goal) at least one of 64 placements drawn
    uniformly over the placement region (yaw uniform) is reached from one of 4 starts.

Random chains (uniform DH parameters) sometimes cannot reach a top-down grasp at table
height at all; such scenes have no solution and are not workload instances.

Point-to-point scenes (workload p2p) are certified when neither the start nor the goal
configuration penetrates a box (zero clutter score: no robot sphere inside an obstacle).

    python tests/golden/make_reachable_seeds.py [--count 64] [--only p2p]
"""
import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2510_07674_amd import synth  # noqa: E402

WORKLOADS = ("tiny", "tower4", "tower10", "p2p")


def reachable(o, prob, kind, target, rng, starts):
    for _ in range(starts):
        q = o.ik_iterate(kind, target, rng.uniform(prob.lo, prob.hi), 100)
        if o.ik_error(kind, target, q) < 1e-4:
            return True
    return False


def certify(name, seed):
    prob, pr, _ = synth.config(name, seed)
    o = oracle.Oracle(prob, pr)
    if prob.mode == synth.MODE_P2P:
        pose = np.zeros((prob.B, 4))
        return o.arm_clutter(prob.q_home, pose, 0, 2) == 0.0 and o.arm_clutter(prob.p2p_goal, pose, 0, 2) == 0.0
    rng = np.random.default_rng([seed, 7])
    for b in range(prob.B):
        if not reachable(o, prob, 0, prob.block_init[b], rng, 32):
            return False
    xl, xh, yl, yh = prob.table
    for b in range(prob.B):
        if prob.mode == synth.MODE_FIXED:
            if not reachable(o, prob, 1, prob.goal[b], rng, 32):
                return False
            continue
        z = (b + 0.5) * prob.h
        ok = False
        for _ in range(64):
            t = np.array([rng.uniform(xl, xh), rng.uniform(yl, yh), z, rng.uniform(-np.pi, np.pi)])
            if reachable(o, prob, 1, t, rng, 4):
                ok = True
                break
        if not ok:
            return False
    return True


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64, help="certified seeds to list per workload")
    ap.add_argument("--only", help="recompute this workload's line and keep the others")
    args = ap.parse_args()
    oracle.build(force=False)
    path = os.path.join(HERE, "reachable_seeds.txt")
    kept = {}
    if args.only and os.path.exists(path):
        for line in open(path):
            if line.strip() and not line.startswith("#"):
                kept[line.split()[0]] = line.strip()
    lines = []
    for name in WORKLOADS:
        if args.only and name != args.only and name in kept:
            lines.append(kept[name])
            continue
        seeds, s = [], 0
        while len(seeds) < args.count:
            if certify(name, s):
                seeds.append(s)
            s += 1
        lines.append(f"{name} " + " ".join(map(str, seeds)))
        print(f"{name}: {len(seeds)} of the first {s} seeds certified", flush=True)
    with open(path, "w") as f:
        f.write("# scene seeds certified feasible by make_reachable_seeds.py (oracle IK; p2p: collision-free ends)\n")
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
