"""Point-to-point (one motion from q_home to a goal configuration) on the GPU against
the FP64 oracle.  Cost parity and teacher-forced Adam steps are parametrised into
test_gpu_parity.py; this file covers the seeding, the whole solve and the entry points
that have no meaning without blocks."""
import numpy as np
import pytest
import torch

from paper_2510_07674_amd import synth
from test_gpu_parity import N, T, f32, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    from paper_2510_07674_amd import spasm
    spasm.load()
    return spasm


def test_p2p_init_parity(sp, orc):
    """Seeds: exact ends, and the intermediate waypoint chosen by the same rule; FP32 and
    FP64 may pick different draws only where their clutter scores tie within rounding."""
    for seed in synth.p2p_seeds()[:3]:
        prob, pr, _ = synth.config("p2p", seed)
        dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
        P, W = 64, 32
        q32 = N(dev.traj_init(None, None, W, seed=5, pose=None, P=P))
        q64 = o.p2p_init(P, W, seed=5)
        assert np.abs(q32[:, 0, 0] - q64[:, 0, 0]).max() <= 1e-6
        assert np.abs(q32[:, 0, -1] - q64[:, 0, -1]).max() <= 1e-6
        m = (W - 1) // 2
        same = np.abs(q32 - q64).max(axis=(1, 2, 3)) <= 2e-6
        pose = np.zeros((prob.B, 4))
        qa, qb = q64[0, 0, 0], q64[0, 0, W - 1]
        for p in np.nonzero(~same)[0]:
            sc = lambda qm: sum(o.arm_clutter(x, pose, 0, 2) for x in (qm, 0.5 * (qa + qm), 0.5 * (qm + qb)))
            assert sc(q32[p, 0, m].astype(np.float64)) <= sc(q64[p, 0, m]) + 1e-4, p
        assert same.mean() >= 0.9
        report(f"p2p init seed {seed}", same=float(same.mean()))


def test_p2p_solve(sp, orc):
    """The whole solve on certified scenes: the best trajectory keeps the exact start and
    goal, repeats bit for bit, and the FP64 oracle agrees on its violation."""
    solved = 0
    seeds = synth.p2p_seeds()[:8]
    for seed in seeds:
        prob, pr, cfg = synth.config("p2p", seed)
        dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
        res, bq, _ = dev.solve(cfg)
        res2, bq2, _ = dev.solve(cfg)
        q = N(bq)
        assert q.shape == (1, cfg.W, 7)
        assert np.abs(q[0, 0] - prob.q_home).max() <= 1e-6 and np.abs(q[0, -1] - prob.p2p_goal).max() <= 1e-6
        keys = ("success", "n_sat", "best", "viol", "cost", "length")
        assert torch.equal(bq, bq2) and all(res[k] == res2[k] for k in keys)
        _, v64, *_ = o.traj_cost(q[None].astype(np.float64), np.zeros((1, prob.B, 4)), 1, grad=False)
        assert abs(v64[0] - res["viol"]) <= 1e-5 + 1e-4 * v64[0]
        solved += int(res["success"])
    report("p2p solve", solved=solved, scenes=len(seeds))
    assert solved >= 1


def test_p2p_rejects_block_entry_points(sp):
    prob, pr, cfg = synth.config("p2p", synth.p2p_seeds()[0])
    dev = sp.Problem(prob, pr)
    with pytest.raises(sp.SpasmError):
        dev.ik_lift(torch.zeros(4, prob.B, 4, device="cuda"), seed=0)
    srv = sp.Server(1 << 28, max_slots=4)
    with pytest.raises(sp.SpasmError):
        srv.submit(dev, cfg, 1)
    srv.close()


@pytest.mark.parametrize("W,P", [(4, 33), (64, 5)])
def test_p2p_smallest_and_largest_W(sp, orc, W, P):
    """One-segment trajectories of 4 and 64 waypoints (one or two waves, ragged lanes):
    cost parity and a solve that keeps its ends."""
    from test_gpu_parity import _traj_parity
    rng = np.random.default_rng(W)
    prob, pr, cfg = synth.config("p2p", synth.p2p_seeds()[3])
    o = orc.Oracle(prob, pr)
    q = o.p2p_init(P, W, seed=2)
    q[:, :, 1:-1] += rng.normal(0, 0.2, size=q[:, :, 1:-1].shape)
    _traj_parity(sp, orc, prob, pr, q, np.zeros((P, prob.B, 4)), f"p2p W{W}")
    dev = sp.Problem(prob, pr)
    cfg = synth.dataclasses.replace(cfg, W=W, M=P)
    res, bq, _ = dev.solve(cfg)
    bq = N(bq)
    assert bq.shape == (1, W, 7)
    assert np.abs(bq[0, 0] - prob.q_home).max() <= 1e-6 and np.abs(bq[0, -1] - prob.p2p_goal).max() <= 1e-6
