"""Serving benchmark: a Poisson stream of mixed solves (blocks U{1..10}, boxes U{0..80},
waypoints {16, 32} per segment, particles scaled with the block count) served by the
continuous-batching server, against the plain path that runs one solve per launch
sequence in arrival order.  Arrival rates are fractions of the plain path's measured
capacity on the same mix.  Latency = completion time - arrival time (wall clock).

    python -m paper_2510_07674_amd.serve_bench --requests 1000 --rates 0.3 0.6 0.9
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import spasm, synth


def make_mix(n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        prob, pr, cfg = synth.serving_request(rng, seed=10_000 + i)
        reqs.append((spasm.Problem(prob, pr), cfg))
    return reqs


def arrivals(n, rate, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def run_plain(reqs, arr):
    """One solve at a time in arrival order (each solve = its own launch sequence)."""
    work = {}
    lat = []
    t0 = time.perf_counter()
    for (dev, cfg), ta in zip(reqs, arr):
        now = time.perf_counter() - t0
        if now < ta:
            time.sleep(ta - now)
        key = (dev.B, cfg.W, cfg.M, cfg.N1)
        if key not in work:
            work[key] = dev.make_workspace(cfg)
        dev.solve(cfg, work[key])
        lat.append(time.perf_counter() - t0 - ta)
        if len(lat) % 250 == 0:
            print(f"plain: {len(lat)} of {len(reqs)} done", flush=True)
    total = time.perf_counter() - t0
    return np.array(lat), total


def run_served(reqs, arr, budget, slots, iters):
    srv = spasm.Server(budget, slots, iters)
    lat = {}
    results = {}
    t0 = time.perf_counter()
    nxt = 0
    n = len(reqs)
    while len(lat) < n:
        now = time.perf_counter() - t0
        while nxt < n and arr[nxt] <= now:
            dev, cfg = reqs[nxt]
            srv.submit(dev, cfg, nxt)
            nxt += 1
        active, pending = srv.step()
        for c in srv.poll():
            lat[c["req_id"]] = time.perf_counter() - t0 - arr[c["req_id"]]
            results[c["req_id"]] = c
            if len(lat) % 250 == 0:
                print(f"served: {len(lat)} of {n} done", flush=True)
        if active == 0 and pending == 0 and nxt < n:
            wait = arr[nxt] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
    total = time.perf_counter() - t0
    srv.close()
    return np.array([lat[i] for i in range(n)]), total, results


def summary(lat, total, n, seed=0):
    """p50 / p99 / mean latency in ms with 95 % bootstrap intervals (2000 resamples of the
    requests), and throughput."""
    ms = lat * 1e3
    rng = np.random.default_rng(seed)
    boot = ms[rng.integers(0, len(ms), size=(2000, len(ms)))]
    ci = lambda v: [float(np.percentile(v, 2.5)), float(np.percentile(v, 97.5))]
    return {"p50_ms": float(np.percentile(ms, 50)), "p50_ci95": ci(np.percentile(boot, 50, axis=1)),
            "p99_ms": float(np.percentile(ms, 99)), "p99_ci95": ci(np.percentile(boot, 99, axis=1)),
            "mean_ms": float(ms.mean()), "mean_ci95": ci(boot.mean(axis=1)), "solves_per_s": n / total}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--rates", type=float, nargs="+", default=[0.3, 0.6, 0.9])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget-gb", type=float, default=8.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--iters-per-step", type=int, default=25)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    reqs = make_mix(args.requests, args.seed)
    # capacity of the plain path on this mix (back-to-back, warm)
    run_plain(reqs[:4], np.zeros(4))
    lat, total = run_plain(reqs, np.zeros(len(reqs)))
    capacity = len(reqs) / total
    out = {"metric": "serving p50/p99 latency (ms) and solves/s, continuous batching vs one solve per launch",
           "mix": "blocks U{1..10}, boxes U{0..80}, W in {16,32}, M=128B, N1=8M, K=50+25B",
           "requests": args.requests, "plain_capacity_solves_per_s": capacity, "rates": []}
    for frac in args.rates:
        rate = frac * capacity
        arr = arrivals(len(reqs), rate, args.seed + int(frac * 1000))
        lp, tp = run_plain(reqs, arr)
        ls, ts, _ = run_served(reqs, arr, int(args.budget_gb * 2**30), args.slots, args.iters_per_step)
        out["rates"].append({"load": frac, "arrival_per_s": rate, "plain": summary(lp, tp, len(reqs)),
                             "served": summary(ls, ts, len(reqs)),
                             "served_all_ok": all(r["status"] == 0 for r in _.values())})
        print(json.dumps(out["rates"][-1]), flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
