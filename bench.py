#!/usr/bin/env python3
"""Benchmark: particle-waypoint cost+grad evals/s of the SPaSM hot path on one MI355X.

One step = one whole solve (stage-1 sampling, scoring, top-M, descent, ordering; lift;
seeding; fused stage-2 Adam descent; final evaluation and best particle) of a 10-block
tower in clutter (80 boxes, 48 spheres, 16384 -> 2048 particles, 20 segments x 32
waypoints, 300 iterations; `--workload tower4` runs the 4-block tower), each step on a
different seeded problem whose description is already on the device.  value = stage-2
particle-waypoint evaluations (each a fused cost + gradient + Adam update) per second of
whole-job time.  The dominant kernel (the fused stage-2 launch) is timed live with HIP
events recorded around it inside spasm_solve, on the solve's stream.
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


def stored_counters(workload):
    """Machine-readable lines of the committed counter summary of the fused stage-2 kernel
    on this workload (profiles/k_traj_<workload>_counters.md), or None when there is none
    or the kernel source or the build flags have changed since the counters were taken
    (the hash covers kernels.hip followed by build.py)."""
    import hashlib
    summary = os.path.join(ROOT, "profiles", f"k_traj_{workload}_counters.md")
    pkg = os.path.join(ROOT, "paper_2510_07674_amd")
    try:
        fields = {}
        for line in open(summary):
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip()
        h = hashlib.sha256()
        for src in (os.path.join(pkg, "csrc", "kernels.hip"), os.path.join(pkg, "build.py")):
            with open(src, "rb") as f:
                h.update(f.read())
        sha = h.hexdigest()
    except OSError:
        return None
    if fields.get("kernels_sha256") != sha or fields.get("workload") != workload:
        return None
    return fields


def stored_traffic(workload):
    """HBM bytes per launch of the fused stage-2 kernel (FETCH_SIZE and WRITE_SIZE scaled
    by a plain copy's readings), or None (see stored_counters)."""
    f = stored_counters(workload)
    return float(f["traffic_bytes_per_launch"]) if f and "traffic_bytes_per_launch" in f else None


def stored_executed_flop(workload):
    """FP32 arithmetic the fused stage-2 kernel executes per launch, from its VALU counters
    (64 lanes x (ADD + MUL + 2 FMA + TRANS) F32 instructions), or None."""
    f = stored_counters(workload)
    return float(f["executed_fp32_flop_per_launch"]) if f and "executed_fp32_flop_per_launch" in f else None


def _oracle_iteration_rate(name, seconds, P=32):
    """Stage-2 particle-waypoint evaluations per second of the FP64 oracle (cost, gradient
    and Adam step) on P particles of the workload's first certified scene, lifted and
    seeded as a solve starts them; iterations repeat until `seconds` have passed."""
    import numpy as np
    import oracle
    from paper_2510_07674_amd import synth
    prob, pr, cfg = synth.config(name, synth.certified_seeds(name)[0])
    o = oracle.Oracle(prob, pr)
    rng = np.random.default_rng(0)
    W = cfg.W
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
    return k * P * 2 * prob.B * W / dt, k, P, dt


def _oracle_solve_extrapolated(name, sub=128):
    """The FP64 oracle's whole solve of the workload's first certified scene at full size,
    extrapolated: stage 1 is run in full; the lift, the seeding and ONE stage-2 iteration
    are run on the first `sub` of the M particles (every particle's work is independent
    and alike) and scaled by M / sub; the iteration is scaled to K iterations (the work
    per iteration is constant)."""
    import oracle
    from paper_2510_07674_amd import synth
    prob, pr, cfg = synth.config(name, synth.certified_seeds(name)[0])
    o = oracle.Oracle(prob, pr)
    sub = min(sub, cfg.M)
    t0 = time.perf_counter()
    for rnd in range(pr.retries + 1):
        x, c1, v1 = o.stage1(cfg.N1, cfg.M, cfg.seed, rnd)
        order, nsat = o.order(c1, v1)
        if nsat > 0:
            break
    pose = o.initial_poses(x[order])[:sub]
    t1 = time.perf_counter()
    qg, qp = o.ik_lift(pose, cfg.seed)
    q = o.traj_init(qg, qp, cfg.W, cfg.seed, pose)
    t2 = time.perf_counter()
    o.stage2(q, pose, 1)
    t3 = time.perf_counter()
    scale = cfg.M / sub
    return {"stage1_s": t1 - t0, "lift_seed_s": scale * (t2 - t1), "iteration_s": scale * (t3 - t2),
            "solve_s_extrapolated": (t1 - t0) + scale * (t2 - t1) + cfg.K * scale * (t3 - t2), "K": cfg.K,
            "sub": sub, "M": cfg.M}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, seconds):
    """The FP64 oracle (plain C, OpenMP over particles) on the host cores: a bounded sample
    of the same workload on every thread OpenMP is given and on one thread (a child
    process with OMP_NUM_THREADS=1), and its whole solve of the first scene at full size
    extrapolated from one stage-2 iteration."""
    import subprocess
    rate, k, P, dt = _oracle_iteration_rate(name, seconds)
    one = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-rate", name,
                          "--cpu-seconds", str(max(2.0, seconds / 2))],
                         env=dict(os.environ, OMP_NUM_THREADS="1"), capture_output=True, text=True, timeout=600)
    rate1 = json.loads(one.stdout.strip().splitlines()[-1])["value"] if one.returncode == 0 else None
    ext = _oracle_solve_extrapolated(name)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": rate, "unit": "evals/s", "cores": cores, "kind": "oracle", "cpu_model": _cpu_model(),
            "value_1core": rate1,
            "sample": f"{k} stage-2 Adam iterations (cost + gradient + Adam, FP64) x {P} particles x "
                      f"{'x'.join(map(str, _shape(name)))} waypoints of {name}'s first scene ({dt:.1f} s, OpenMP over "
                      f"particles on {cores} threads; value_1core: the same on one thread)",
            "solve_s_extrapolated": ext["solve_s_extrapolated"],
            "solve_extrapolation": f"{name} at full size: stage 1 {ext['stage1_s']:.2f} s (run in full) + lift and "
                                   f"seeding {ext['lift_seed_s']:.2f} s + {ext['K']} x {ext['iteration_s']:.2f} s per "
                                   f"stage-2 iteration; lift, seeding and one iteration timed on {ext['sub']} of the "
                                   f"{ext['M']} particles and scaled, the iteration extrapolated linearly to K"}


def _shape(name):
    from paper_2510_07674_amd import synth
    prob, _, cfg = synth.config(name, synth.certified_seeds(name)[0])
    return 2 * prob.B, cfg.W


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tower10", choices=["tower10", "tower4", "tiny"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--oracle-rate", metavar="WORKLOAD", help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (hardware-counter scale)")
    args = ap.parse_args()
    if args.oracle_rate:  # the CPU baseline's one-thread leg (a child process, no GPU)
        rate, _, _, _ = _oracle_iteration_rate(args.oracle_rate, args.cpu_seconds)
        print(json.dumps({"value": rate}), flush=True)
        return
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
    executed = stored_executed_flop(args.workload)
    kind = "tower" if prob.mode == synth.MODE_TOWER else "fixed-goal"
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
        "config": {"workload": f"{args.workload}: {prob.B}-block {kind}, {prob.O} boxes, {prob.S} spheres, "
                               f"N1={cfg.N1} -> M={cfg.M}, {2 * prob.B}x{cfg.W} waypoints, K={cfg.K}",
                   "blocks": prob.B, "obstacles": prob.O, "spheres": prob.S, "N1": cfg.N1, "M": cfg.M,
                   "segments": 2 * prob.B, "W": cfg.W, "K": cfg.K,
                   "scenes": f"seeds {seeds[args.warmup:]} (timed)",
                   "generator": "seeded random 7-DOF DH chains (a U[0,0.1] m, d U[0,0.35] m, twists +-pi/2 on "
                                "joints 1-6 and {-pi/2,0,pi/2} on joint 7, limits +-2.8 rad), 6-7 spheres per "
                                "link r U[0.03,0.08] m, 5 cm cube blocks; AABB boxes of sides U[0.05,0.3] m "
                                "uniform on a 1x1 m table, kept only if they clear by 1 cm a plan that solves the "
                                "box-free scene (feasible by construction; start q_home pinned)"},
        "pct_fp32_peak": 100.0 * value * F / PEAK_FP32,
        "pct_fp32_peak_kind": "dense-equivalent: algorithmic FLOP of every sphere-box pair (the broad and "
                              "narrow phases skip most of them) per second of whole-job time",
        "flop_per_eval": F,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "stage1_ms_mean": float(np.mean([r["stage1_ms"] for r in results])),
        "stage2_ms_mean": float(np.mean([r["stage2_ms"] for r in results])),
        "success_rate": float(np.mean([r["success"] for r in results])),
        "roofline": {"bound": "alu", "kernel": "k_traj<2> (fused stage-2 cost+grad+Adam)",
                     "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": stored_traffic(args.workload), "avg_ms": opt_ms,
                     "executed_fp32": None if executed is None else {
                         "tflops": executed / (opt_ms * 1e-3) / 1e12,
                         "frac": executed / (opt_ms * 1e-3) / PEAK_FP32,
                         "flop_per_launch": executed,
                         "source": f"profiles/k_traj_{args.workload}_counters.md (VALU F32 counters, 64 lanes, "
                                   f"FMA = 2)"}},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
