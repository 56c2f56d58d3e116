#!/usr/bin/env python3
"""Benchmark: particle-waypoint cost+grad evals/s of the SPaSM hot path on one MI355X.

One step = one whole solve (stage-1 sampling, scoring, top-M, descent, ordering; lift;
seeding; fused stage-2 Adam descent; final evaluation and best particle) of a 4-block
tower in clutter (40 boxes, 4096 -> 1024 particles, 8 segments x 32 waypoints, 200
iterations), each step on a different seeded problem whose description is already on
the device.  value = stage-2 particle-waypoint evaluations (each a fused cost +
gradient + Adam update) per second of whole-job time.  The dominant kernel (the fused
stage-2 launch) is timed live with HIP events recorded around it inside spasm_solve.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12   # MI355X FP32 vector peak (FLOP/s)


def flop_per_eval(S, O, B, W):
    """Algorithmic FLOPs of one particle-waypoint evaluation (cost + gradient + update).
    Counting add/sub/mul 1, fma 2, transcendental 1, min/max/compare/select 0:
    505 forward kinematics, 18 per sphere centre, 9 per sphere-box test, 18 per
    sphere-block (yawed box) test, held block (transfer interior) 144 + 72 per target,
    450 for the reverse pass, limits, smoothness and the Adam update."""
    b_vis = (B - 1) + 0.5 * (W - 1) / W
    f_tr = (W - 2) / (2.0 * W)
    return 505 + 18 * S + 9 * S * O + 18 * S * b_vis + f_tr * (144 + 72 * (O + B - 1)) + 450


def stored_traffic(workload):
    """HBM bytes per launch of the fused stage-2 kernel from the committed counter summary,
    or None when the kernel source has changed since the counters were taken or the
    workload is not the one they were taken on."""
    import hashlib
    summary = os.path.join(ROOT, "profiles", "k_traj_tower4_counters.md")
    src = os.path.join(ROOT, "paper_2510_07674_amd", "csrc", "kernels.hip")
    try:
        fields = {}
        for line in open(summary):
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip()
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if fields.get("kernels_sha256") != sha or fields.get("workload") != workload:
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(name, seconds):
    """The FP64 oracle (OpenMP over particles) on a bounded sample of the same workload:
    stage-2 cost + gradient + Adam steps on 32 particles of the first problem."""
    import numpy as np
    import oracle
    from paper_2510_07674_amd import synth
    prob, pr, cfg = synth.config(name, 0)
    o = oracle.Oracle(prob, pr)
    rng = np.random.default_rng(0)
    P, W = 32, cfg.W
    x = synth.clustered_placements(rng, prob, P, spread=0.01)
    pose = o.initial_poses(x)
    qg, qp = o.ik_lift(pose, seed=0)
    q = o.traj_init(qg, qp, W, seed=0, pose=pose)
    mq, vq, mp, vp = (np.zeros_like(q), np.zeros_like(q), np.zeros_like(pose), np.zeros_like(pose))
    k, t0 = 0, time.perf_counter()
    while True:
        k += 1
        phase, lr = o.schedule(k, pr.k_lin2(cfg.K), pr.eta2, pr.alpha2)
        _, _, gq, gp, _, _ = o.traj_cost(q, pose, phase)
        q, pose, mq, vq, mp, vp = o.adam_step(q, pose, mq, vq, mp, vp, gq, gp, lr, k)
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    evals = k * P * 2 * prob.B * W
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": evals / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} stage-2 Adam iterations x {P} particles x {2 * prob.B}x{W} waypoints of {name} seed 0 "
                      f"({dt:.1f} s, FP64, OpenMP over particles)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tower4")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (hardware-counter scale)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        torch.cuda.set_device(0)
        n = args.copy_calibration << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (particles are independent, "
              f"a multi-GPU run would shard them with no per-iteration exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2510_07674_amd import spasm, synth

    torch.cuda.set_device(0)
    n = args.warmup + args.steps
    seeds = synth.certified_seeds(args.workload)
    seeds = [seeds[i % len(seeds)] for i in range(n)]
    probs = []
    for s in seeds:
        prob, pr, cfg = synth.config(args.workload, s)
        probs.append(spasm.Problem(prob, pr))
    dev0 = probs[0]
    work = dev0.make_workspace(cfg)
    best_q = torch.empty(2 * prob.B, cfg.W, 7, device="cuda")
    best_pose = torch.empty(prob.B, 4, device="cuda")
    for i in range(args.warmup):
        probs[i].solve(cfg, work, best_q, best_pose)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for i in range(args.warmup, n):
        res, _, _ = probs[i].solve(cfg, work, best_q, best_pose)
        results.append(res)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    evals_per_solve = cfg.M * 2 * prob.B * cfg.W * cfg.K
    F = flop_per_eval(prob.S, prob.O, prob.B, cfg.W)
    value = args.steps * evals_per_solve / wall
    lat = np.array([r["total_ms"] for r in results])
    opt_ms = float(np.mean([r["opt_ms"] for r in results]))
    achieved = F * evals_per_solve / (opt_ms * 1e-3)
    line = {
        "metric": "particle-waypoint cost+grad evals/s (%FP32 peak); p50/p99 solve latency ms",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {prob.B}-block tower, {prob.O} boxes, {prob.S} spheres, "
                               f"N1={cfg.N1} -> M={cfg.M}, {2 * prob.B}x{cfg.W} waypoints, K={cfg.K}",
                   "blocks": prob.B, "obstacles": prob.O, "spheres": prob.S, "N1": cfg.N1, "M": cfg.M,
                   "segments": 2 * prob.B, "W": cfg.W, "K": cfg.K},
        "pct_fp32_peak": 100.0 * value * F / PEAK_FP32,
        "flop_per_eval": F,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "stage1_ms_mean": float(np.mean([r["stage1_ms"] for r in results])),
        "stage2_ms_mean": float(np.mean([r["stage2_ms"] for r in results])),
        "success_rate": float(np.mean([r["success"] for r in results])),
        "roofline": {"bound": "alu", "kernel": "k_traj<2> (fused stage-2 cost+grad+Adam)",
                     "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": stored_traffic(args.workload), "avg_ms": opt_ms},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
