"""Workload definition: the feasible-by-construction tower and fixed-goal scenes
(tests/golden/witness_scenes.txt) and the point-to-point seeds
(tests/golden/reachable_seeds.txt) are reproducible from their certificate scripts, the
plan each scene was built around solves it with zero violation (every penetration exactly
zero), and excluded scenes really fail the certificate."""
import importlib.util
import os

import numpy as np
import pytest

from paper_2510_07674_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _script(name):
    spec = importlib.util.spec_from_file_location(name, os.path.join(HERE, "golden", name + ".py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_p2p_seeds_reproduce(orc):
    cert = _script("make_reachable_seeds")
    seeds = synth.certified_seeds("p2p")
    assert len(seeds) >= 32 and seeds == sorted(set(seeds))
    for s in seeds[:2]:
        assert cert.certify("p2p", s)
    first_gap = next(s for s in range(seeds[-1]) if s not in seeds)
    assert not cert.certify("p2p", first_gap)


@pytest.mark.parametrize("name", ["tiny", "tower4"])
def test_witness_scenes_reproduce_and_are_solved(orc, name):
    """The first listed scene: the plan is rebuilt, the accepted boxes are the recorded
    ones, and in the finished scene the plan's violation is zero except for the grasp and
    tie residuals of the exact IK (below 1e-9 m); the first seed missing from the list is
    rejected by the certificate."""
    mk = _script("make_witness_scenes")
    scenes = synth.witness_scenes(name)
    seeds = sorted(scenes)
    assert len(seeds) >= 32
    s = seeds[0]
    prob0, q, pose = mk.build_plan(name, s)
    assert mk.accept_boxes(name, s, prob0, q, pose) == scenes[s]
    prob, pr, cfg = synth.config(name, s)
    B, O, S, mode = synth.SCENES[name]
    assert prob.O == O and prob.B == B and q.shape == (2 * B, cfg.W, 7)
    o = orc.Oracle(prob, pr)
    cat = o.traj_residuals(q[None], pose[None])[0]
    assert np.all(cat[[0, 1, 2, 3, 6, 7]] == 0.0) and np.all(cat[[4, 5]] < 1e-9)
    c, v, *_ = o.traj_cost(q[None], pose[None], orc.QUAD, grad=False)
    assert v[0] < 1e-9
    # the plan starts at the robot's start configuration
    assert np.array_equal(q[0, 0], np.clip(prob.q_home, prob.lo, prob.hi))
    first_gap = next(v for v in range(seeds[-1]) if v not in scenes)
    assert mk.certify(name, first_gap) is None


@pytest.mark.parametrize("name", ["tetris5", "tetris8"])
def test_packing_pieces_tile_the_box(name):
    """Every packing instance: pieces of 1..8 cells, each 4-connected, that together
    cover the box's grid exactly once at the recorded packing."""
    for seed in range(20):
        prob, _, _ = synth.config(name, seed)
        a = prob.h
        x0, x1, y0, y1 = prob.table
        cols, rows = round((x1 - x0) / a), round((y1 - y0) / a)
        seen = np.zeros((rows, cols), dtype=int)
        for b in range(prob.B):
            n = int(prob.pack_cells[b])
            assert 1 <= n <= synth.MAX_CELLS
            cx, cy, yaw = prob.pack_solution[b]
            assert yaw == 0.0
            cells = set()
            for k in range(n):
                c = round((cx + prob.pack_off[b, k, 0] - x0) / a - 0.5)
                r = round((cy + prob.pack_off[b, k, 1] - y0) / a - 0.5)
                seen[r, c] += 1
                cells.add((r, c))
            assert not prob.pack_off[b, n:].any()
            # flood fill from one cell reaches all of the piece
            todo, reach = [next(iter(cells))], set()
            while todo:
                r, c = todo.pop()
                if (r, c) in reach:
                    continue
                reach.add((r, c))
                todo += [(r + dr, c + dc) for dr, dc in ((1, 0), (-1, 0), (0, 1), (0, -1)) if (r + dr, c + dc) in cells]
            assert reach == cells
        assert (seen == 1).all()
