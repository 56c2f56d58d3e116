"""Writes witness_scenes.txt: scenes of the named solve workloads (tiny, tower4, tower10)
that are feasible by construction, built with the FP64 oracle (test infrastructure).

For scene seed s the chain, spheres, blocks and goals (or hidden tower site) are drawn
by synth.make_problem without boxes.  A plan that solves that box-free scene exactly is
then built:

  * placements: fixed goals as given; a tower stacks block b at the site at its slot
    height (b + 1/2) h, with the first yaw of a short list that the arm reaches;
  * grasp and place configurations: damped least-squares IK from the previous
    configuration and from uniform starts, run until the error is below 1e-11; among the
    solutions that touch no block, the nearest first;
  * each motion segment: W waypoints along a joint-space polyline, the first of these
    shapes whose segment has zero violation in the box-free scene (checked at the W
    waypoints and at four sub-steps between each pair of them): the straight line; lines
    through a perturbed midpoint; an RRT-Connect path (shortcut, corners kept as
    waypoints) whose nodes and edges (every 0.02 rad) have zero violation, at most 12
    RRT-Connect runs of 800 iterations per block.

The plan's violation is zero (grasp and tie residuals below 1e-9) with every penetration
exactly zero.  The scene's boxes are then the first O of synth.candidate_boxes(s, ...)
whose clearance from the plan (robot spheres at every sub-step, the held block inside
transfers, every block at its initial pose and at its placement) is at least 1 cm.
Seeds for which no plan is found, or fewer than O candidates of the first 50 O fit, are
not instances.  The file lists, per workload and seed, the accepted candidate indices.

    python tests/golden/make_witness_scenes.py [--only tower4] [--jobs 8]

Instances listed: 32 tiny, 32 tower4 and 16 tower10 scenes (the 10-block plans are slow
to build: about one seed in five has one).
"""
import argparse
import dataclasses
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2510_07674_amd import synth  # noqa: E402

FINE = 4          # sub-steps per waypoint interval in the plan checks
CLEAR = 0.01      # boxes clear the plan by this much (m)
EXACT = 1e-11     # IK error accepted as exact
W_OF = {"tiny": 16, "tower4": 32, "tower10": 32}
YAWS = (0.0, math.pi / 2, -math.pi / 2, math.pi, math.pi / 4, -math.pi / 4, 3 * math.pi / 4, -3 * math.pi / 4)


def segment(qa, qb, qm, W):
    """W waypoints from qa to qb, straight lines through qm at index (W-1)/2."""
    m = (W - 1) // 2
    out = np.empty((W, 7))
    for w in range(W):
        if w <= m:
            out[w] = qa + (w / m) * (qm - qa) if m > 0 else qa
        else:
            out[w] = qm + ((w - m) / (W - 1 - m)) * (qb - qm)
    out[0], out[-1] = qa, qb
    return out


def refine(seg, f=FINE):
    """The same polyline with f sub-steps per interval: (W-1) f + 1 waypoints."""
    rows = [seg[0]]
    for w in range(len(seg) - 1):
        for k in range(1, f + 1):
            rows.append(seg[w] + (seg[w + 1] - seg[w]) * (k / f))
    rows[-1] = seg[-1]
    return np.array(rows)


def ik_solutions(o, prob, kind, target, q_pref, rng, starts=40, iters=400):
    """Exact IK solutions (error < EXACT) from q_pref and uniform starts, nearest first."""
    sols = []
    for q0 in [q_pref] + [rng.uniform(prob.lo, prob.hi) for _ in range(starts)]:
        q = o.ik_iterate(kind, target, q0, iters)
        if o.ik_error(kind, target, q) < EXACT and not any(np.abs(q - s).max() < 1e-6 for s in sols):
            sols.append(q)
    sols.sort(key=lambda q: float(np.linalg.norm(q - q_pref)))
    return sols


def segment_ok(o, prob, NS, s, fine, pose):
    """Zero violation on every slot of segment s (grasp / tie residuals below 1e-9)."""
    q = np.repeat(fine[None, None], NS, axis=1)
    r = o.traj_slot_residuals(q, pose[None])[0, s]
    hard = r[:, [0, 1, 2, 3, 6]].max()
    return hard == 0.0 and r[:, 4].max() < 1e-9 and r[:, 5].max() < 1e-9


def polyline(points, W):
    """W waypoints along the joint-space polyline through `points`, evenly by length,
    with the first and last points exact."""
    pts = np.asarray(points)
    seg = np.linalg.norm(np.diff(pts, axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    if cum[-1] == 0.0:
        return np.repeat(pts[:1], W, axis=0)
    out = np.empty((W, 7))
    for w in range(W):
        t = cum[-1] * w / (W - 1)
        k = min(int(np.searchsorted(cum, t, side="right")) - 1, len(seg) - 1)
        f = (t - cum[k]) / seg[k] if seg[k] > 0 else 0.0
        out[w] = pts[k] + f * (pts[k + 1] - pts[k])
    out[0], out[-1] = pts[0], pts[-1]
    return out


def lifted(o, prob, q, dz):
    """A configuration whose block frame sits dz above q's, held upright (IK from q), or
    None when the arm does not reach it exactly."""
    F = o.fk(q)
    R, p = F[8, :9].reshape(3, 3), F[8, 9:]
    G = prob.grasp
    t = p - R @ (G[:, :3].T @ G[:, 3])
    tgt = np.array([t[0], t[1], t[2] + dz, 0.0])
    r = o.ik_iterate(0, tgt, q, 200)
    return r if o.ik_error(0, tgt, r) < 1e-6 else None


def interior_ok(o, NS, s, qa, qb, pts, pose):
    """Zero violation of each configuration of pts [n, 7] as an interior waypoint of segment
    s (which blocks it meets, whether it holds one) between the ends qa and qb."""
    fine = np.concatenate([qa[None], pts, qb[None]])
    q = np.repeat(fine[None, None], NS, axis=1)
    r = o.traj_slot_residuals(q, pose[None])[0, s, 1:-1]
    return r[:, [0, 1, 2, 3, 6]].max(axis=1) == 0.0


def edge_points(a, b, res=0.02):
    n = max(1, int(math.ceil(np.abs(b - a).max() / res)))
    return a[None] + (b - a)[None] * (np.arange(1, n + 1) / n)[:, None]


def rrt_connect(o, prob, NS, s, qa, qb, pose, rng, iters=800, step=0.25):
    """A collision-free joint-space path qa -> qb for the interior of segment s by
    RRT-Connect (Kuffner and LaValle, 2000), shortcut, or None."""
    def free_edge(a, b):
        return bool(interior_ok(o, NS, s, qa, qb, edge_points(a, b), pose).all())

    trees = [[qa], [qb]]
    parent = [[-1], [-1]]
    for it in range(iters):
        A, Bt = (0, 1) if it % 2 == 0 else (1, 0)
        x = rng.uniform(prob.lo, prob.hi)
        ta = np.array(trees[A])
        i = int(np.argmin(np.abs(ta - x).max(axis=1)))
        d = x - ta[i]
        n = np.abs(d).max()
        y = ta[i] + (d if n <= step else d * (step / n))
        if not free_edge(ta[i], y):
            continue
        trees[A].append(y)
        parent[A].append(i)
        # connect the other tree towards y
        tb = np.array(trees[Bt])
        j = int(np.argmin(np.abs(tb - y).max(axis=1)))
        z = tb[j]
        while True:
            d = y - z
            n = np.abs(d).max()
            if n <= step:
                if free_edge(z, y):
                    trees[Bt].append(y)
                    parent[Bt].append(j)
                    j = len(trees[Bt]) - 1
                    # join the two branches at y
                    def branch(t, k):
                        out = []
                        while k >= 0:
                            out.append(trees[t][k])
                            k = parent[t][k]
                        return out
                    pa, pb = branch(A, len(trees[A]) - 1), branch(Bt, j)
                    path = (pa[::-1] + pb[1:]) if A == 0 else (pb[::-1] + pa[1:])
                    return shortcut(free_edge, path, rng)
                break
            w = z + d * (step / n)
            if not free_edge(z, w):
                break
            trees[Bt].append(w)
            parent[Bt].append(j)
            j = len(trees[Bt]) - 1
            z = w
    return None


def shortcut(free_edge, path, rng, tries=60):
    path = list(path)
    for _ in range(tries):
        if len(path) <= 2:
            break
        i, j = sorted(rng.choice(len(path), 2, replace=False))
        if j - i >= 2 and free_edge(path[i], path[j]):
            path = path[:i + 1] + path[j:]
    return path


def corner_polyline(points, W):
    """W waypoints on the polyline through `points` with every corner a waypoint: each
    piece gets at least one interval, the rest spread by length.  None when there are
    more corners than waypoints."""
    pts = np.asarray(points)
    L = np.linalg.norm(np.diff(pts, axis=0), axis=1)
    k = len(L)
    if k > W - 1:
        return None
    n = np.ones(k, int)
    extra = W - 1 - k
    if extra:
        share = L / max(L.sum(), 1e-12) * extra
        n += np.floor(share).astype(int)
        rem = extra - (n.sum() - k)
        for i in np.argsort(-(share - np.floor(share)))[:rem]:
            n[i] += 1
    rows = [pts[0]]
    for i in range(k):
        for t in range(1, n[i] + 1):
            rows.append(pts[i] + (pts[i + 1] - pts[i]) * (t / n[i]))
    out = np.array(rows)
    out[-1] = pts[-1]
    return out


class Budget:
    """RRT-Connect runs left for one block (a work bound, so the output does not depend
    on the machine)."""

    def __init__(self, n):
        self.n = n


def find_segment(o, prob, NS, s, qa, qb, W, pose, rng, budget, tries=30):
    """A segment qa -> qb of W waypoints whose refined polyline has zero violation: the
    straight line, lines through a perturbed midpoint, then (while the budget lasts) an
    RRT-Connect path with its corners kept as waypoints."""
    shapes = [[qa, qb]]
    for k in range(tries):
        shapes.append([qa, np.clip(0.5 * (qa + qb) + 0.5 * rng.uniform(-1, 1, 7), prob.lo, prob.hi), qb])
    for pts in shapes:
        seg = polyline(pts, W)
        if segment_ok(o, prob, NS, s, refine(seg), pose):
            return seg
    for _ in range(2):
        if budget.n <= 0:
            break
        budget.n -= 1
        path = rrt_connect(o, prob, NS, s, qa, qb, pose, rng)
        if path is None:
            continue
        seg = corner_polyline(path, W)
        if seg is not None and segment_ok(o, prob, NS, s, refine(seg), pose):
            return seg
    return None


def build_plan(name, seed):
    """(problem without boxes, q [2B, W, 7], pose [B, 4]) solving the box-free scene, or None."""
    B, O, S, mode = synth.SCENES[name]
    W = W_OF[name]
    prob = synth.witness_problem(name, seed, boxes_idx=[])
    pr = synth.Params()
    o = oracle.Oracle(prob, pr)
    rng = np.random.default_rng([seed, B, 0x7717])
    NS = 2 * B
    qh = np.clip(prob.q_home, prob.lo, prob.hi)
    pose = np.zeros((B, 4))
    # placements beyond the block being planned sit at their initial poses' footprint height
    # until planned (they are not yet visible as placed blocks to earlier segments)
    q = np.zeros((NS, W, 7))
    prev = qh
    for b in range(B):
        # grasp configurations that touch no block, not even the one grasped, so that the
        # approach (where that block is an obstacle) can end next to them; nearest first
        grasps = [g for g in ik_solutions(o, prob, 0, prob.block_init[b], prev, rng, starts=64)
                  if o.arm_clutter(g, pose, b, 2) == 0.0][:6]
        if mode == synth.MODE_FIXED:
            targets = [prob.goal[b]]
        else:
            z = (b + 0.5) * prob.h
            targets = [np.array([prob.site[0], prob.site[1], z, y]) for y in YAWS]
        done = False
        budget = Budget(12)
        # the transit to a grasp does not see block b's placement: find it once per grasp
        transits = [(qg, find_segment(o, prob, NS, 2 * b, prev, qg, W, pose, rng, budget)) for qg in grasps]
        for tgt in targets:
            pose[b] = tgt
            for qg, tr in transits:
                if tr is None:
                    continue
                places = [p for p in ik_solutions(o, prob, 1, tgt, qg, rng, starts=48)
                          if o.arm_clutter(p, pose, b, 1) == 0.0][:4]
                for qp in places:
                    tf = find_segment(o, prob, NS, 2 * b + 1, qg, qp, W, pose, rng, budget)
                    if tf is not None:
                        q[2 * b], q[2 * b + 1] = tr, tf
                        prev, done = qp, True
                        break
                if done:
                    break
            if done:
                break
        if not done:
            return None
    # the whole plan, every slot, at W and refined
    fine = np.stack([refine(q[s]) for s in range(NS)])
    for qq in (q, fine):
        cat = o.traj_residuals(qq[None], pose[None])[0]
        if cat[[0, 1, 2, 3, 6, 7]].max() != 0.0 or cat[[4, 5]].max() >= 1e-9:
            return None
    return prob, q, pose


def accept_boxes(name, seed, prob, q, pose):
    """Indices of the first O candidates that clear the refined plan by CLEAR."""
    B, O, S, mode = synth.SCENES[name]
    cand = synth.candidate_boxes(seed, B, O, S, mode, 50 * O)
    o = oracle.Oracle(prob, synth.Params())
    fine = np.stack([refine(q[s]) for s in range(q.shape[0])])
    clear = o.box_clearance(fine, pose, cand)
    idx = [int(i) for i in np.nonzero(clear >= CLEAR)[0][:O]]
    return idx if len(idx) == O else None


def certify(name, seed):
    """Accepted candidate indices of scene `seed`, or None when it is not an instance."""
    plan = build_plan(name, seed)
    if plan is None:
        return None
    prob, q, pose = plan
    idx = accept_boxes(name, seed, prob, q, pose)
    if idx is None:
        return None
    # the finished scene: the plan is a solution with zero violation
    full = synth.witness_problem(name, seed, boxes_idx=idx)
    o = oracle.Oracle(full, synth.Params())
    cat = o.traj_residuals(q[None], pose[None])[0]
    assert cat[[0, 1, 2, 3, 6, 7]].max() == 0.0 and cat[[4, 5]].max() < 1e-9, (name, seed, cat)
    return idx


def witness(name, seed):
    """(problem with its boxes, q, pose) of a listed scene: the plan rebuilt (deterministic)."""
    prob, q, pose = build_plan(name, seed)
    return synth.witness_problem(name, seed), q, pose


def _work(args):
    name, seed = args
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    return name, seed, certify(name, seed)


COUNT = {"tiny": 32, "tower4": 32, "tower10": 16}  # instances listed per workload


def _write(path, lines):
    lines = sorted(lines, key=lambda ln: (synth.WITNESS_WORKLOADS.index(ln.split()[0]), int(ln.split()[1])))
    with open(path, "w") as f:
        f.write("# workload seed accepted-candidate-box indices; written by make_witness_scenes.py (FP64 oracle)\n")
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", help="recompute this workload's lines and keep the others")
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--max-seeds", type=int, default=400, help="seeds tried per workload at most")
    args = ap.parse_args()
    oracle.build(force=False)
    path = os.path.join(HERE, "witness_scenes.txt")
    lines = []
    if os.path.exists(path):
        lines = [ln.rstrip("\n") for ln in open(path) if ln.strip() and not ln.startswith("#")]
    import multiprocessing as mp
    for name in synth.WITNESS_WORKLOADS:
        if args.only and name != args.only:
            continue
        found, s = [], 0
        with mp.Pool(args.jobs) as pool:
            while len(found) < COUNT[name] and s < args.max_seeds:
                batch = [(name, v) for v in range(s, s + 2 * args.jobs)]
                s += 2 * args.jobs
                for _, seed, idx in pool.imap(_work, batch):
                    if idx is not None and len(found) < COUNT[name]:
                        found.append((seed, idx))
                print(f"{name}: {len(found)} scenes from the first {s} seeds", flush=True)
        lines = [ln for ln in lines if ln.split()[0] != name]
        lines += [f"{name} {seed} " + " ".join(map(str, idx)) for seed, idx in found]
        _write(path, lines)


if __name__ == "__main__":
    main()
