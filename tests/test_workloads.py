"""Workload definition: the certified scene seeds (tests/golden/reachable_seeds.txt) are
reproducible from the certificate script, and excluded scenes really fail it."""
import importlib.util
import os

import numpy as np
import pytest

from paper_2510_07674_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _certificate():
    spec = importlib.util.spec_from_file_location("make_reachable_seeds",
                                                  os.path.join(HERE, "golden", "make_reachable_seeds.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_certified_seeds_reproduce(orc):
    cert = _certificate()
    for name in ("tiny", "tower4", "tower10", "p2p"):
        seeds = synth.certified_seeds(name)
        assert len(seeds) >= 32 and seeds == sorted(set(seeds))
        for s in seeds[:2]:
            assert cert.certify(name, s)
        first_gap = next(s for s in range(seeds[-1]) if s not in seeds)
        assert not cert.certify(name, first_gap)


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
