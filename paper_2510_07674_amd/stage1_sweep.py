"""Placement-only (stage 1) sweep over sampling batch N and optimisation batch M, the
paper's hyperparameter ablation (Sec. IV, N in 2^[9,19], M in 2^[8,13]) rerun on the
synthetic towers-in-clutter and on the synthetic packing (Tetris) workloads: for each
(N, M) and each trial, placement rounds (spasm_place_round) repeat until one satisfies;
the time to that first feasible placement is wall clock on the host, including the
per-round check of the satisfying count.

    python -m paper_2510_07674_amd.stage1_sweep --workload tower4 --trials 20
    python -m paper_2510_07674_amd.stage1_sweep --workload tetris5 --nlist 9 11 13 15 --mlist 8 10 12
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import spasm, synth


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="tower4")
    ap.add_argument("--trials", type=int, default=20)
    ap.add_argument("--max-rounds", type=int, default=64)
    ap.add_argument("--nlog", type=int, nargs=2, default=[9, 19])
    ap.add_argument("--mlog", type=int, nargs=2, default=[8, 13])
    ap.add_argument("--nlist", type=int, nargs="*", help="log2 N values (overrides --nlog)")
    ap.add_argument("--mlist", type=int, nargs="*", help="log2 M values (overrides --mlog)")
    ap.add_argument("--tuning-seeds", action="store_true",
                    help="packing workloads: draw scenes from seeds 1000.. (disjoint from the instances 0..99)")
    ap.add_argument("--param", nargs="*", default=[], metavar="NAME=VALUE",
                    help="override stage-1 parameters of the workload, e.g. eta1=0.01 k_lin1=50")
    args = ap.parse_args()
    nlogs = args.nlist or list(range(args.nlog[0], args.nlog[1] + 1))
    mlogs = args.mlist or list(range(args.mlog[0], args.mlog[1] + 1))
    torch.cuda.set_device(0)
    if args.tuning_seeds:
        if not args.workload.startswith("tetris"):
            raise SystemExit("tuning seeds are defined for the packing workloads only")
        seeds = list(range(1000, 1000 + args.trials))
    else:
        seeds = synth.instance_seeds(args.workload)[: args.trials]
    problems = []
    for s in seeds:
        prob, pr, _ = synth.config(args.workload, s)
        for kv in args.param:
            k, v = kv.split("=")
            setattr(pr, k, type(getattr(pr, k))(v))
        problems.append(spasm.Problem(prob, pr))
    nsat_host = torch.empty(1, dtype=torch.int32, pin_memory=True)
    rows = []
    for nl in nlogs:
        for ml in mlogs:
            N, M = 1 << nl, 1 << ml
            if M > N:
                continue
            work = problems[0].place_workspace(N, M)
            # warm-up (kernel loading, allocator)
            problems[0].place_round(N, M, seed=10_000, rnd=0, work=work)
            torch.cuda.synchronize()
            times, rounds, solved = [], [], 0
            for t, dev in enumerate(problems):
                t0 = time.perf_counter()
                r = 0
                while r < args.max_rounds:
                    _, _, _, nsat = dev.place_round(N, M, seed=seeds[t], rnd=r, work=work)
                    nsat_host.copy_(nsat, non_blocking=True)
                    torch.cuda.synchronize()
                    r += 1
                    if int(nsat_host[0]) > 0:
                        solved += 1
                        break
                times.append(time.perf_counter() - t0)
                rounds.append(r)
            row = {"N": N, "M": M, "mean_ms": 1e3 * float(np.mean(times)),
                   "ci95_ms": 1e3 * 1.96 * float(np.std(times, ddof=1)) / np.sqrt(len(times)) if len(times) > 1 else 0.0,
                   "p50_ms": 1e3 * float(np.median(times)),
                   "mean_rounds": float(np.mean(rounds)), "solved": solved, "trials": len(problems)}
            rows.append(row)
            print(json.dumps(row), flush=True)
    best = min(rows, key=lambda r: r["mean_ms"] if r["solved"] == r["trials"] else float("inf"))
    print(json.dumps({"metric": "time to first feasible placement (stage 1 only), mean over trials",
                      "workload": args.workload, "params": args.param, "trials": len(problems), "best": best}),
          flush=True)


if __name__ == "__main__":
    main()
