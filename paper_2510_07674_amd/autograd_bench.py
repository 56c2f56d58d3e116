"""Forward + backward throughput of the stage-2 cost as a torch.autograd.Function
(`spasm.SpasmCost`: cost-only kernel forward, hand-written adjoint kernel backward) on a
batch of 256 particles x 8 segments x 32 waypoints = 65,536 particle-waypoints of the
4-block tower, started where the solver starts them (one placement round, lift, seeding).

    python -m paper_2510_07674_amd.autograd_bench --reps 50
"""
from __future__ import annotations

import argparse
import json

import torch

from . import spasm, synth


def solver_start(dev, prob, cfg, P, seed):
    """Placements of one stage-1 round lifted and seeded as the solver does."""
    x, _, _, _ = dev.place_round(cfg.N1, P, seed=seed, rnd=0)
    B = prob.B
    pose = torch.zeros(P, B, 4, device="cuda")
    pose[..., 0] = x[..., 0]
    pose[..., 1] = x[..., 1]
    pose[..., 2] = (torch.arange(B, device="cuda", dtype=torch.float32) + 0.5) * prob.h
    pose[..., 3] = x[..., 2]
    qg, qp = dev.ik_lift(pose, seed)
    return dev.traj_init(qg, qp, cfg.W, seed, pose), pose


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="tower4")
    ap.add_argument("--particles", type=int, default=256)
    ap.add_argument("--reps", type=int, default=50)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    seed = synth.certified_seeds(args.workload)[0]
    prob, pr, cfg = synth.config(args.workload, seed)
    dev = spasm.Problem(prob, pr)
    q0, pose0 = solver_start(dev, prob, cfg, args.particles, seed)
    q = q0.clone().requires_grad_(True)
    pose = pose0.clone().requires_grad_(True)
    pw = q.shape[0] * q.shape[1] * q.shape[2]

    def fwd():
        return spasm.SpasmCost.apply(q, pose, dev, spasm.PHASE_LIN)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for _ in range(3):
        fwd().sum().backward()
    torch.cuda.synchronize()
    t_f = t_b = 0.0
    for _ in range(args.reps):
        q.grad = None
        pose.grad = None
        ev[0].record()
        cost = fwd()
        ev[1].record()
        cost.sum().backward()
        ev[2].record()
        torch.cuda.synchronize()
        t_f += ev[0].elapsed_time(ev[1])
        t_b += ev[1].elapsed_time(ev[2])
    t_f /= args.reps
    t_b /= args.reps
    print(json.dumps({
        "metric": "SpasmCost forward + backward, particle-waypoints/s",
        "workload": args.workload, "particles": q.shape[0], "particle_waypoints": pw,
        "forward_ms": t_f, "backward_ms": t_b, "fwd_bwd_ms": t_f + t_b,
        "fwd_bwd_per_s": pw / ((t_f + t_b) * 1e-3), "reps": args.reps,
    }), flush=True)


if __name__ == "__main__":
    main()
