"""Seeded synthetic workloads: towers in clutter on a random 7-DOF serial chain.

This module only draws random problem descriptions (robot model, collision
spheres, box clutter, blocks, skeleton, solver parameters).  It contains none of
the method's arithmetic: no kinematics, no distances, no costs, no sampling of
particles.  Both the FP64 oracle and the HIP path consume what it returns.

The paper's own scenes (Sec. IV-C, Fig. "tower stacking", Table III) are not
available; these synthetic towers-in-clutter stand in for them:

* chain: classic DH, a ~ U[0, 0.1] m, d ~ U[0, 0.35] m, joint limits +-2.8 rad, base
  at the world origin with z up, tool offset 0.10 m along the last joint axis; twists
  alpha ~ U{-pi/2, +pi/2} on joints 1-6 and U{-pi/2, 0, +pi/2} on joint 7 (a zero twist
  makes two consecutive axes parallel, and such chains rarely hold a block upright on
  the table);
* robot spheres (the paper represents the robot as spheres, Sec. III): spread
  evenly by arc length along each link's polyline, radius ~ U[0.03, 0.08] m;
* cube blocks of edge 0.05 m resting at random table poses, top-down grasp;
* a 1 x 1 m table centred on the robot base (table top z = 0); blocks, goals and
  the tower live in a placement region in front of the robot, 0.2-0.55 m out;
* axis-aligned box obstacles with sides ~ U[0.05, 0.3] m resting on the table;
* the named solve workloads (tiny, tower4, tower10) are feasible by construction: their
  boxes are the first O of a seeded sequence of candidate boxes (uniform over the table)
  that clear, by at least 1 cm, a plan that solves the box-free scene exactly (built
  offline by tests/golden/make_witness_scenes.py with the FP64 oracle); this module only
  reads the list of accepted candidates (`witness_scenes`) and draws the candidates;
* other scenes (the serving mix) keep their boxes out of a square around the base and
  small squares around the blocks' initial poses and a hidden tower site.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

N_JOINTS = 7
TABLE = (-0.5, 0.5, -0.5, 0.5)           # clutter table x_lo, x_hi, y_lo, y_hi; top at z = 0
REGION = (0.2, 0.55, -0.35, 0.35)        # placement region (the problem's bounding box)

MODE_TOWER = 0                           # block b goes to tower slot b (heights (b+1/2) h)
MODE_FIXED = 1                           # block b goes to a given fixed pose
MODE_PACK = 2                            # polyomino pieces packed into the region (stage 1 only)
MODE_P2P = 3                             # one motion from q_home to p2p_goal (trajectory only)
MAX_CELLS = 8                            # cells per packing piece

# weight order shared by every consumer of Params.weights()
WEIGHT_NAMES = ("stable", "height", "coll", "start", "tie", "arm", "block", "lim", "smooth")


@dataclasses.dataclass
class Problem:
    dh: np.ndarray            # (7, 3) float64: a, d, alpha per joint
    lo: np.ndarray            # (7,) joint lower limits
    hi: np.ndarray            # (7,) joint upper limits
    tool_d: float             # tool offset along the last joint axis
    q_home: np.ndarray        # (7,) start configuration (pinned)
    sph_link: np.ndarray      # (S,) int32, link index 1..7, non-decreasing
    sph_c: np.ndarray         # (S, 3) centre in the link frame
    sph_r: np.ndarray         # (S,) radius
    boxes: np.ndarray         # (O, 6) centre xyz, half extents xyz (axis aligned)
    h: float                  # block edge
    block_init: np.ndarray    # (B, 4) x, y, z, yaw of the initial block poses
    mode: int                 # MODE_TOWER or MODE_FIXED
    goal: np.ndarray          # (B, 4) fixed goal poses (MODE_FIXED); tower: slot poses, xy unused
    grasp: np.ndarray         # (3, 4) rigid transform G, block frame -> end-effector frame
    table: np.ndarray         # (4,) placement region x_lo, x_hi, y_lo, y_hi
    block_margin: float = 1e-3  # block collision spheres have radius h/4 - block_margin
    # packing pieces (MODE_PACK): piece b is the union of pack_cells[b] square cells of edge
    # h centred at pack_off[b, k] in the piece frame; the region is the packing box
    pack_cells: np.ndarray = None   # (B,) int32, 1..MAX_CELLS
    pack_off: np.ndarray = None     # (B, MAX_CELLS, 2) float64, unused rows zero
    pack_solution: np.ndarray = None  # (B, 3) one exact packing (x, y, yaw), for tests
    sample_yaw_steps: int = 0       # stage-1 yaw samples: 0 uniform, n > 0 on n directions
    p2p_goal: np.ndarray = None     # (7,) goal configuration (MODE_P2P; the start is q_home)
    site: np.ndarray = None         # (2,) the hidden tower site kept clear of clutter (MODE_TOWER)

    @property
    def S(self) -> int:
        return int(self.sph_r.shape[0])

    @property
    def O(self) -> int:
        return int(self.boxes.shape[0])

    @property
    def B(self) -> int:
        return int(self.block_init.shape[0])


@dataclasses.dataclass
class Params:
    # cost weights (the paper only says "scalar weights"): constraint terms dominate the
    # smoothness objective so that the solution is feasible.  Squared residuals (height,
    # grasp, tie) carry large weights so that near the 1e-3 success threshold their
    # gradients are comparable with the unit-weight linear penetration terms.
    w_stable: float = 10.0
    w_height: float = 1000.0
    w_coll: float = 1.0
    w_start: float = 100.0
    w_tie: float = 100.0
    w_arm: float = 1.0
    w_block: float = 1.0
    w_lim: float = 1.0
    w_smooth: float = 1e-3
    # stage 1: plain gradient descent, linear phase with eta_k = eta1 (1 - k/k_lin1),
    # then k_quad1 quadratic steps at alpha1
    k_lin1: int = 25
    k_quad1: int = 5
    eta1: float = 0.01
    alpha1: float = 0.5
    # stage 2: Adam under the same schedule shape; k_lin2 = round(lin_frac2 * K)
    lin_frac2: float = 5.0 / 6.0
    eta2: float = 1e-2
    alpha2: float = 2e-4
    beta1: float = 0.9
    beta2: float = 0.999
    # Adam's epsilon at the gradient a 1 mm grasp or tie residual produces (2 w r |J| ~ 0.1):
    # smaller gradients take plain-descent steps instead of normalised ones, so the exactly
    # lifted grasp and place configurations are not thrown off by the first steps
    adam_eps: float = 0.1
    # lift / initialisation
    ik_iters: int = 50
    ik_restarts: int = 8      # multi-start lift: starts per (particle, block)
    mid_candidates: int = 8   # seeding: intermediate-waypoint draws per segment
    ik_lambda: float = 0.05
    ik_noise: float = 0.5
    mid_noise: float = 0.5
    # success test and stage-1 retries
    sat_eps: float = 1e-3
    retries: int = 4
    # augmented-Lagrangian outer loop of stage 2 (Sec. III-B): every al_every iterations
    # the grasp and tie multipliers step by al_rho * 2w * residual; 0 = plain penalties
    al_every: int = 0
    al_rho: float = 1.0

    def weights(self) -> np.ndarray:
        return np.array([getattr(self, "w_" + n) for n in WEIGHT_NAMES], dtype=np.float64)

    def k_lin2(self, K: int) -> int:
        return int(round(self.lin_frac2 * K))


# stage-1 schedule of the packing workloads (the paper tunes it per problem): twice the
# towers' descent steps (50 linear + 10 quadratic) and a smaller quadratic step, chosen
# by time to the first exact packing on the GPU over tuning scenes (seeds 1000..), which
# are disjoint from the instances 0..99
PACK_PARAMS = Params(eta1=0.01, alpha1=0.1, k_lin1=50, k_quad1=10)


@dataclasses.dataclass
class SolveConfig:
    N1: int          # stage-1 samples (0: fixed goals, no stage 1)
    M: int           # particles kept after stage 1 = stage-2 particles
    W: int           # waypoints per motion segment
    K: int           # stage-2 iterations
    seed: int = 0


def _chain(rng: np.random.Generator):
    a = rng.uniform(0.0, 0.1, N_JOINTS)
    d = rng.uniform(0.0, 0.35, N_JOINTS)
    alpha = np.concatenate([rng.choice(np.array([-math.pi / 2, math.pi / 2]), N_JOINTS - 1),
                            rng.choice(np.array([-math.pi / 2, 0.0, math.pi / 2]), 1)])
    dh = np.stack([a, d, alpha], axis=1)
    # limits rounded to FP32-representable values: both precisions then compare the same
    # numbers, so the limit hinges switch at the same configuration
    lo = np.full(N_JOINTS, float(np.float32(-2.8)))
    hi = np.full(N_JOINTS, float(np.float32(2.8)))
    return dh, lo, hi


def _spheres(rng: np.random.Generator, dh: np.ndarray, S: int):
    """Spread S spheres over the 7 links (first links get the remainder), evenly by arc
    length along each link's polyline in its own frame: the previous joint origin
    (-a, -d sin(alpha), -d cos(alpha)), the foot of the common normal (-a, 0, 0), and
    the link origin (0, 0, 0)."""
    per = [S // N_JOINTS + (1 if k < S % N_JOINTS else 0) for k in range(N_JOINTS)]
    links, cents = [], []
    for k in range(N_JOINTS):
        a, d, al = dh[k]
        p0 = np.array([-a, -d * math.sin(al), -d * math.cos(al)])
        p1 = np.array([-a, 0.0, 0.0])
        p2 = np.zeros(3)
        l0 = float(np.linalg.norm(p1 - p0))
        l1 = float(np.linalg.norm(p2 - p1))
        tot = l0 + l1
        for m in range(per[k]):
            s = (m + 0.5) / per[k] * tot
            if tot <= 0.0:
                c = p2.copy()
            elif s <= l0:
                c = p0 + (p1 - p0) * (s / l0)
            else:
                c = p1 + (p2 - p1) * ((s - l0) / l1)
            links.append(k + 1)
            cents.append(c)
    r = rng.uniform(0.03, 0.08, S)
    return np.array(links, dtype=np.int32), np.array(cents), r


def _keep_out(cx, cy, hx, hy, pts, rad):
    for (px, py) in pts:
        if abs(cx - px) < hx + rad and abs(cy - py) < hy + rad:
            return True
    return False


def make_problem(seed: int, B: int, O: int, S: int = 42, mode: int = MODE_TOWER,
                 h: float = 0.05, boxes: np.ndarray = None) -> Problem:
    """Draw one seeded problem.  Deterministic in (seed, B, O, S, mode, h).  With `boxes`
    given ([n, 6]) those are the obstacles and O only seeds the draw."""
    rng = np.random.default_rng([seed, B, O, S, mode, 0x5A5A])
    dh, lo, hi = _chain(rng)
    sph_link, sph_c, sph_r = _spheres(rng, dh, S)
    xlo, xhi, ylo, yhi = REGION
    edge = 0.03

    # initial block poses: separated discs in the placement region
    pts = []
    for _ in range(100000):
        if len(pts) == B:
            break
        p = (rng.uniform(xlo + edge, xhi - edge), rng.uniform(ylo + edge, yhi - edge))
        if all((p[0] - q[0]) ** 2 + (p[1] - q[1]) ** 2 > 0.08 ** 2 for q in pts):
            pts.append(p)
    if len(pts) < B:
        raise ValueError("cannot place %d blocks in the placement region" % B)
    yaw = rng.uniform(-math.pi, math.pi, B)
    block_init = np.array([[pts[i][0], pts[i][1], h / 2, yaw[i]] for i in range(B)])

    keep = list(pts)
    goal = np.zeros((B, 4))
    if mode == MODE_FIXED:
        for i in range(B):
            for _ in range(100000):
                g = (rng.uniform(xlo + edge, xhi - edge), rng.uniform(ylo + edge, yhi - edge))
                if all((g[0] - q[0]) ** 2 + (g[1] - q[1]) ** 2 > 0.12 ** 2 for q in keep):
                    break
            keep.append(g)
            goal[i] = [g[0], g[1], h / 2, rng.uniform(-math.pi, math.pi)]
    else:
        for _ in range(1000):  # hidden tower site, kept free of clutter
            g = (rng.uniform(xlo + 0.05, xhi - 0.05), rng.uniform(ylo + 0.05, yhi - 0.05))
            if all((g[0] - q[0]) ** 2 + (g[1] - q[1]) ** 2 > 0.08 ** 2 for q in keep):
                break
        keep.append(g)
        for i in range(B):
            goal[i] = [math.nan, math.nan, (i + 0.5) * h, math.nan]

    site = np.array(g, dtype=np.float64) if mode != MODE_FIXED else None
    if boxes is not None:
        return _finish(dh, lo, hi, sph_link, sph_c, sph_r, np.asarray(boxes, dtype=np.float64).reshape(-1, 6), h,
                       block_init, mode, goal, site)
    boxes = []
    tries = 0
    while len(boxes) < O and tries < 100000:
        tries += 1
        half = rng.uniform(0.05, 0.3, 3) / 2
        cx = rng.uniform(TABLE[0], TABLE[1])
        cy = rng.uniform(TABLE[2], TABLE[3])
        if _keep_out(cx, cy, half[0], half[1], [(0.0, 0.0)], 0.2):
            continue
        if _keep_out(cx, cy, half[0], half[1], keep, 0.08):
            continue
        boxes.append([cx, cy, half[2], half[0], half[1], half[2]])
    boxes = np.array(boxes, dtype=np.float64).reshape(-1, 6)
    return _finish(dh, lo, hi, sph_link, sph_c, sph_r, boxes, h, block_init, mode, goal, site)


def _finish(dh, lo, hi, sph_link, sph_c, sph_r, boxes, h, block_init, mode, goal, site) -> Problem:
    # top-down grasp: end effector at the top-face centre, its z axis pointing down
    grasp = np.array([[1.0, 0.0, 0.0, 0.0],
                      [0.0, -1.0, 0.0, 0.0],
                      [0.0, 0.0, -1.0, h / 2]])
    return Problem(dh=dh, lo=lo, hi=hi, tool_d=0.10, q_home=np.zeros(N_JOINTS),
                   sph_link=sph_link, sph_c=sph_c, sph_r=sph_r, boxes=boxes, h=h,
                   block_init=block_init, mode=mode, goal=goal, grasp=grasp,
                   table=np.array(REGION, dtype=np.float64), site=site)


def candidate_boxes(seed: int, B: int, O: int, S: int, mode: int, n: int) -> np.ndarray:
    """The first n of a scene's seeded sequence of candidate boxes: sides U[0.05, 0.3] m,
    centre uniform over the table, resting on it.  [n, 6] centre, half extents."""
    rng = np.random.default_rng([seed, B, O, S, mode, 0xB0C5])
    u = rng.uniform(size=(n, 5))  # one row per candidate: the first k rows do not depend on n
    half = (0.05 + 0.25 * u[:, :3]) / 2
    cx = TABLE[0] + (TABLE[1] - TABLE[0]) * u[:, 3]
    cy = TABLE[2] + (TABLE[3] - TABLE[2]) * u[:, 4]
    return np.stack([cx, cy, half[:, 2], half[:, 0], half[:, 1], half[:, 2]], axis=1)


def _partition(rng: np.random.Generator, rows: int, cols: int, B: int) -> np.ndarray:
    """Random partition of a rows x cols grid into B 4-connected pieces of near-equal size
    (grown from random seed cells, one random frontier cell at a time; redrawn when a
    piece gets boxed in).  Returns the owner index of every cell."""
    n = rows * cols
    sizes = [n // B + (1 if k < n % B else 0) for k in range(B)]
    if max(sizes) > MAX_CELLS:
        raise ValueError("pieces of more than %d cells" % MAX_CELLS)
    for _ in range(10000):
        owner = -np.ones((rows, cols), dtype=np.int64)
        start = rng.choice(n, B, replace=False)
        count = [1] * B
        for k, c in enumerate(start):
            owner[c // cols, c % cols] = k
        stuck = False
        while any(count[k] < sizes[k] for k in range(B)):
            grow = []
            for k in range(B):
                if count[k] >= sizes[k]:
                    continue
                front = set()
                for (r, c) in zip(*np.nonzero(owner == k)):
                    for dr, dc in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                        rr, cc = r + dr, c + dc
                        if 0 <= rr < rows and 0 <= cc < cols and owner[rr, cc] < 0:
                            front.add((int(rr), int(cc)))
                if front:
                    grow.append((k, sorted(front)))
            if not grow:
                stuck = True
                break
            k, front = grow[int(rng.integers(len(grow)))]
            r, c = front[int(rng.integers(len(front)))]
            owner[r, c] = k
            count[k] += 1
        if not stuck:
            return owner
    raise ValueError("no partition found")


def make_packing(seed: int, B: int, rows: int, cols: int, cell: float = 0.04) -> Problem:
    """Draw one seeded packing problem (the paper's Tetris task, Sec. IV, with synthetic
    pieces): the rows x cols box of square cells (edge `cell`) is cut into B connected
    polyominoes that fill it without gaps, so every exact packing uses all of the space.
    The robot part is drawn as for the towers (the packing cost does not use it).  Piece
    frames sit at the centroid of their cells; initial poses are a row of spots outside
    the box.  Stage-1 yaw samples are quarter turns: exact packings of square cells only
    exist there."""
    rng = np.random.default_rng([seed, B, rows, cols, 0x7E7A])
    base = make_problem(seed, B=1, O=0, S=42, mode=MODE_TOWER, h=cell)
    owner = _partition(rng, rows, cols, B)
    xc = 0.5 * (REGION[0] + REGION[1])
    x0, y0 = xc - 0.5 * cols * cell, -0.5 * rows * cell
    n_cells = np.zeros(B, dtype=np.int32)
    off = np.zeros((B, MAX_CELLS, 2))
    sol = np.zeros((B, 3))
    for k in range(B):
        rr, cc = np.nonzero(owner == k)
        cx = x0 + (cc + 0.5) * cell
        cy = y0 + (rr + 0.5) * cell
        ox, oy = float(cx.mean()), float(cy.mean())
        n_cells[k] = len(cx)
        off[k, : len(cx), 0] = cx - ox
        off[k, : len(cx), 1] = cy - oy
        sol[k] = [ox, oy, 0.0]
    yaw = rng.uniform(-math.pi, math.pi, B)
    block_init = np.array([[-0.3 + 0.6 * (k + 0.5) / B, -0.4, cell / 2, yaw[k]] for k in range(B)])
    goal = np.zeros((B, 4))
    goal[:, :] = math.nan
    goal[:, 2] = cell / 2
    region = np.array([x0, x0 + cols * cell, y0, y0 + rows * cell])
    return dataclasses.replace(base, boxes=np.zeros((0, 6)), h=cell, block_init=block_init, mode=MODE_PACK,
                               goal=goal, table=region, pack_cells=n_cells, pack_off=off, pack_solution=sol,
                               sample_yaw_steps=4)


def make_p2p(seed: int, O: int = 20, S: int = 42) -> Problem:
    """Draw one seeded point-to-point problem (the paper's motion-planning use, Sec. IV,
    with synthetic scenes in place of MotionBenchMaker): a random chain and spheres as for
    the towers, O boxes on the table as clutter, a start (q_home) and a goal configuration
    uniform within the joint limits.  The single block of the description is a
    placeholder that the trajectory cost does not use.  Instances whose start or goal is
    in collision are dropped by the certificate in tests/golden (p2p_seeds)."""
    base = make_problem(seed, B=1, O=O, S=S, mode=MODE_FIXED)
    rng = np.random.default_rng([seed, O, S, 0x9292])
    lo, hi = base.lo, base.hi
    q0 = rng.uniform(lo, hi)
    q1 = rng.uniform(lo, hi)
    return dataclasses.replace(base, q_home=q0, mode=MODE_P2P, p2p_goal=q1,
                               goal=np.array([[math.nan, math.nan, base.h / 2, math.nan]]))


_GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")
_SEEDS_FILE = os.path.join(_GOLDEN, "reachable_seeds.txt")
_WITNESS_FILE = os.path.join(_GOLDEN, "witness_scenes.txt")
WITNESS_WORKLOADS = ("tiny", "tower4", "tower10")
# (B, O, S, mode) of the scenes of each named solve workload
SCENES = {"tiny": (1, 10, 42, MODE_FIXED), "tower4": (4, 40, 42, MODE_TOWER), "tower10": (10, 80, 48, MODE_TOWER)}


def witness_scenes(name: str) -> dict:
    """{seed: accepted candidate-box indices} of a workload's feasible-by-construction
    scenes (list written by tests/golden/make_witness_scenes.py)."""
    out = {}
    with open(_WITNESS_FILE) as f:
        for line in f:
            parts = line.split()
            if parts and parts[0] == name:
                out[int(parts[1])] = [int(v) for v in parts[2:]]
    if not out:
        raise KeyError(name)
    return out


def witness_problem(name: str, seed: int, boxes_idx=None) -> Problem:
    """Scene `seed` of a named solve workload: the seeded chain, spheres and blocks with
    the accepted candidate boxes (`boxes_idx`, default: the recorded ones; [] = no boxes).
    A seed that is not listed gives a scene of the same sizes whose boxes are only kept out
    of the squares around the base, blocks and tower site (not certified feasible; parity
    tests use such scenes too)."""
    B, O, S, mode = SCENES[name]
    if boxes_idx is None:
        listed = witness_scenes(name)
        if seed not in listed:
            return make_problem(seed, B=B, O=O, S=S, mode=mode)
        boxes_idx = listed[seed]
    idx = list(boxes_idx)
    n = max(idx) + 1 if idx else 0
    boxes = candidate_boxes(seed, B, O, S, mode, n)[idx] if idx else np.zeros((0, 6))
    return make_problem(seed, B=B, O=O, S=S, mode=mode, boxes=boxes)


def certified_seeds(name: str) -> list:
    """Scene seeds of a workload.  tiny, tower4, tower10: the scenes built around a plan
    that solves them (witness_scenes), in seed order; p2p: the seeds whose start and goal
    are collision-free (list written by tests/golden/make_reachable_seeds.py)."""
    if name in WITNESS_WORKLOADS:
        return sorted(witness_scenes(name))
    with open(_SEEDS_FILE) as f:
        for line in f:
            parts = line.split()
            if parts and parts[0] == name:
                return [int(v) for v in parts[1:]]
    raise KeyError(name)


def instance_seeds(name: str) -> list:
    """Scene seeds of a workload: the certified list for the tower workloads (their
    instances depend on the robot reaching every block), seeds 0..99 for the packing
    workloads (stage 1 only)."""
    if name.startswith("tetris"):
        return list(range(100))
    return certified_seeds(name)


def p2p_seeds() -> list:
    """Point-to-point scene seeds whose start and goal are collision-free (list written by
    tests/golden/make_p2p_seeds.py)."""
    return certified_seeds("p2p")


# The five workloads.  C1..C3 are solve configurations, C4 is the differentiable-cost
# batch, C5 is the serving mix (sizes drawn per request).
def config(name: str, seed: int = 0):
    """Return (problem, params, solve_config) for a named workload."""
    if name == "tiny":           # 1 block to a fixed target, 10 boxes, 2 x 16 waypoints
        prob = witness_problem(name, seed)
        return prob, Params(), SolveConfig(N1=0, M=64, W=16, K=50, seed=seed)
    if name == "tower4":         # 4-block tower, 40 boxes, 8 x 32 waypoints
        prob = witness_problem(name, seed)
        return prob, Params(), SolveConfig(N1=4096, M=1024, W=32, K=200, seed=seed)
    if name == "tower10":        # 10-block tower, 80 boxes, 20 x 32 waypoints, 48 spheres
        prob = witness_problem(name, seed)
        return prob, Params(), SolveConfig(N1=16384, M=2048, W=32, K=300, seed=seed)
    if name == "p2p":            # one motion between two configurations among 20 boxes
        prob = make_p2p(seed, O=20)
        return prob, Params(), SolveConfig(N1=0, M=256, W=32, K=100, seed=seed)
    if name == "tetris5":        # 5 pieces of 4 cells packed into a 4 x 5 box (stage 1 only)
        prob = make_packing(seed, B=5, rows=4, cols=5)
        return prob, dataclasses.replace(PACK_PARAMS), SolveConfig(N1=4096, M=1024, W=32, K=0, seed=seed)
    if name == "tetris8":        # 8 pieces of 4 cells packed into a 4 x 8 box (stage 1 only)
        prob = make_packing(seed, B=8, rows=4, cols=8)
        return prob, dataclasses.replace(PACK_PARAMS), SolveConfig(N1=16384, M=2048, W=32, K=0, seed=seed)
    raise KeyError(name)


def serving_request(rng: np.random.Generator, seed: int):
    """One request of the serving mix: blocks U{1..10}, obstacles U{0..80},
    waypoints {16, 32} per segment, particle counts scaled with the block count."""
    B = int(rng.integers(1, 11))
    O = int(rng.integers(0, 81))
    W = int(rng.choice([16, 32]))
    P2 = int(min(max(128 * B, 128), 2048))
    prob = make_problem(seed, B=B, O=O, S=42)
    return prob, Params(), SolveConfig(N1=8 * P2, M=P2, W=W, K=50 + 25 * B, seed=seed)


def random_states(rng: np.random.Generator, prob: Problem, P: int, W: int):
    """Random stage-2 states for cost/gradient parity: joint angles uniform within
    the limits (slightly beyond, so the limit hinge is exercised), block poses uniform
    over the table at the tower slot heights with small height noise."""
    B = prob.B
    span = prob.hi - prob.lo
    q = rng.uniform(prob.lo - 0.05 * span, prob.hi + 0.05 * span, size=(P, 2 * B, W, N_JOINTS))
    pose = np.empty((P, B, 4))
    xlo, xhi, ylo, yhi = prob.table
    pose[..., 0] = rng.uniform(xlo, xhi, size=(P, B))
    pose[..., 1] = rng.uniform(ylo, yhi, size=(P, B))
    if prob.mode == MODE_FIXED:
        pose[..., 2] = prob.goal[None, :, 2]
    else:
        pose[..., 2] = (np.arange(B) + 0.5)[None, :] * prob.h + rng.normal(0, 0.01, size=(P, B))
    pose[..., 3] = rng.uniform(-math.pi, math.pi, size=(P, B))
    return q, pose


def random_placements(rng: np.random.Generator, prob: Problem, N: int):
    """Random stage-1 states (x, y, yaw per block) uniform over the table."""
    B = prob.B
    xlo, xhi, ylo, yhi = prob.table
    x = np.empty((N, B, 3))
    x[..., 0] = rng.uniform(xlo, xhi, size=(N, B))
    x[..., 1] = rng.uniform(ylo, yhi, size=(N, B))
    x[..., 2] = rng.uniform(-math.pi, math.pi, size=(N, B))
    return x


def clustered_placements(rng: np.random.Generator, prob: Problem, N: int, spread: float = 0.03):
    """Stage-1 states with the blocks stacked near one random spot, so that the
    stability and block-block terms are active."""
    B = prob.B
    xlo, xhi, ylo, yhi = prob.table
    x = np.empty((N, B, 3))
    cx = rng.uniform(xlo + 0.1, xhi - 0.1, size=(N, 1))
    cy = rng.uniform(ylo + 0.1, yhi - 0.1, size=(N, 1))
    x[..., 0] = cx + rng.normal(0, spread, size=(N, B))
    x[..., 1] = cy + rng.normal(0, spread, size=(N, B))
    x[..., 2] = rng.uniform(-math.pi, math.pi, size=(N, B))
    return x


def near_packing(rng: np.random.Generator, prob: Problem, N: int, spread: float = 0.004,
                 yaw_spread: float = 0.05):
    """Stage-1 states of a packing problem scattered around its exact packing (Gaussian
    noise on x, y and yaw), so that the cell-cell and wall contacts are active and shallow."""
    x = np.repeat(prob.pack_solution[None], N, axis=0).copy()
    x[..., :2] += rng.normal(0, spread, size=(N, prob.B, 2))
    x[..., 2] += rng.normal(0, yaw_spread, size=(N, prob.B))
    return x
