"""Time to first solution of the whole method (the paper's solve-time measure) on the
listed synthetic scenes: spasm_solve_ttfs with a success check every `check_every`
stage-2 iterations and up to `attempts` attempts with fresh samples.  Reports the
configuration-space length of the returned path too (the paper's second measure for
its motion-planning comparison).

    python -m paper_2510_07674_amd.ttfs_bench --workload tower4 --solves 20
    python -m paper_2510_07674_amd.ttfs_bench --workload p2p --solves 31 --check-every 10
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import spasm, synth


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="tower4")
    ap.add_argument("--solves", type=int, default=20)
    ap.add_argument("--check-every", type=int, default=25)
    ap.add_argument("--attempts", type=int, default=4)
    ap.add_argument("--param", nargs="*", default=[], metavar="NAME=VALUE",
                    help="override solver parameters, e.g. al_every=10 al_rho=0.1")
    ap.add_argument("--K", type=int, help="override the stage-2 iteration count")
    ap.add_argument("--M", type=int, help="override the particle count (stage-1 samples scale with it, N1 = 8 M)")
    ap.add_argument("--first", type=int, default=0, help="start at this position of the certified seed list")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    seeds = synth.certified_seeds(args.workload)[args.first: args.first + args.solves + 1]
    rows = []
    for i, s in enumerate(seeds):
        prob, pr, cfg = synth.config(args.workload, s)
        for kv in args.param:
            k, v = kv.split("=")
            setattr(pr, k, type(getattr(pr, k))(v))
        if args.K is not None:
            cfg = synth.dataclasses.replace(cfg, K=args.K)
        if args.M is not None:
            cfg = synth.dataclasses.replace(cfg, M=args.M, N1=8 * args.M if cfg.N1 else 0)
        res, _, _ = spasm.Problem(prob, pr).solve_ttfs(cfg, args.check_every, args.attempts)
        if i == 0:
            continue  # warm-up
        rows.append({"seed": s, "ms": res["total_ms"], "success": bool(res["success"]), "attempts": res["attempts"],
                     "iters": res["iters"], "viol": res["viol"], "length": res["length"]})
        print(json.dumps(rows[-1]), flush=True)
    ok = [r for r in rows if r["success"]]
    ms = np.array([r["ms"] for r in ok]) if ok else np.array([np.nan])
    print(json.dumps({"metric": "time to first solution (ms), solved instances", "workload": args.workload,
                      "params": args.param, "M": args.M, "K": args.K,
                      "check_every": args.check_every, "max_attempts": args.attempts, "solves": len(rows),
                      "solved": len(ok), "p50_ms": float(np.percentile(ms, 50)), "p90_ms": float(np.percentile(ms, 90)),
                      "mean_ms": float(ms.mean()),
                      "mean_ci95_ms": float(1.96 * ms.std(ddof=1) / np.sqrt(len(ms))) if len(ms) > 1 else None,
                      "mean_iters_solved": float(np.mean([r["iters"] for r in ok])) if ok else None,
                      "mean_length_solved": float(np.mean([r["length"] for r in ok])) if ok else None}),
          flush=True)


if __name__ == "__main__":
    main()
