import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


def scara_problem(B=1, O=0, seed=0, S=28):
    """A hand-built chain whose end effector always points straight down and whose
    spheres all sit at least 2 cm above the top of any block on the table:
    joint 1 vertical (d = 0.3), two horizontal links, a flip (alpha = pi) so the
    remaining axes point down, a 0.15 m drop, then short horizontal links.  With the
    0.10 m tool the end effector is at z = 0.05 = block top for every configuration."""
    from paper_2510_07674_amd import synth
    dh = np.array([[0.0, 0.3, 0.0],
                   [0.35, 0.0, 0.0],
                   [0.3, 0.0, math.pi],
                   [0.05, 0.15, 0.0],
                   [0.05, 0.0, 0.0],
                   [0.05, 0.0, 0.0],
                   [0.0, 0.0, 0.0]])
    rng = np.random.default_rng(seed)
    link, cen, rad = synth._spheres(rng, dh, S)
    # keep spheres of the descending link 4 only on its upper part so the lowest
    # sphere bottom stays above z = 0.07
    rad = np.minimum(rad, 0.08)
    boxes = np.zeros((O, 6))
    return synth.Problem(dh=dh, lo=np.full(7, -2.8), hi=np.full(7, 2.8), tool_d=0.10,
                         q_home=np.zeros(7), sph_link=link, sph_c=cen, sph_r=rad, boxes=boxes,
                         h=0.05, block_init=np.zeros((B, 4)), mode=synth.MODE_FIXED,
                         goal=np.zeros((B, 4)), grasp=np.array([[1.0, 0, 0, 0], [0, -1.0, 0, 0],
                                                                [0, 0, -1.0, 0.025]]),
                         table=np.array(synth.REGION))
