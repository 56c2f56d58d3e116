"""GPU parity of the packing (Tetris) placement path against the FP64 oracle, through the
C ABI.  Same tolerances as the tower parity tests (per particle |c32 - c64| <= 1e-4 |c64|
+ 1e-6, gradients in L2 with the same floor; states whose oracle kink margin is below
1e-5 m are left out of the gradient comparison).  The yaw direction index of quarter-turn
samples is compared exactly."""
import math

import numpy as np
import pytest
import torch

from paper_2510_07674_amd import synth
from test_gpu_parity import ABS, KINK, REL, N, T, check_cost, check_grad, f32, report

N_ = N  # N is also a particle count below

pytestmark = pytest.mark.gpu

PACK = ["tetris5", "tetris8"]


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    from paper_2510_07674_amd import spasm
    spasm.load()
    return spasm


@pytest.mark.parametrize("name", PACK)
def test_pack_sample_matches_oracle(sp, orc, name):
    prob, pr, _ = synth.config(name, 3)
    dev = sp.Problem(prob, pr)
    x32 = N(dev.sample(4000, seed=21, rnd=1))
    x64 = orc.Oracle(prob, pr).sample(4000, 21, 1)
    assert np.abs(x32[..., :2] - x64[..., :2]).max() <= 1e-6
    j32 = np.round((x32[..., 2] + math.pi) / (math.pi / 2)).astype(int)
    j64 = np.round((x64[..., 2] + math.pi) / (math.pi / 2)).astype(int)
    assert np.array_equal(j32, j64) and set(np.unique(j64)) == {0, 1, 2, 3}
    assert np.abs(x32[..., 2] - x64[..., 2]).max() <= 1e-6
    report("pack sample " + name, max_abs=float(np.abs(x32 - x64).max()))


@pytest.mark.parametrize("name", PACK)
@pytest.mark.parametrize("phase", [0, 1])
def test_pack_cost_parity(sp, orc, name, phase):
    rng = np.random.default_rng(200 + phase)
    prob, pr, _ = synth.config(name, 4)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    x = np.concatenate([synth.near_packing(rng, prob, 600), synth.random_placements(rng, prob, 400),
                        prob.pack_solution[None]])
    x = f32(x)
    c32, v32, g32 = (N(t) for t in dev.place_cost(T(x), phase))
    c64, v64, g64, kink = o.place_cost(x, phase)
    check_cost(f"pack {name} ph{phase}", c32, c64, v32, v64)
    keep = np.broadcast_to((kink >= KINK)[:, None], g64.shape[:2])
    assert keep.mean() > 0.5, keep.mean()
    check_grad(f"pack {name} ph{phase}", g32, g64, keep)
    c0, v0, _ = (N(t) if t is not None else None for t in dev.place_cost(T(x), phase, grad=False))
    assert np.allclose(c0, c32, rtol=1e-6, atol=1e-7) and np.allclose(v0, v32, rtol=1e-6, atol=1e-7)
    # the exact packing (last row) costs nothing beyond FP32 rounding
    assert c32[-1] < 1e-5 and v32[-1] < 1e-5


def test_pack_cost_full_batch(sp, orc):
    """The 8-piece workload's whole first sample batch (N1 = 16384), as the solver scores
    it.  Costs and violations only: quarter-turn samples are exactly aligned, where the
    yaw derivative of |sin| of the relative yaw is undefined (every sample sits on that
    kink), so their gradients are compared in test_pack_cost_parity on perturbed states."""
    prob, pr, cfg = synth.config("tetris8", 0)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    xs = dev.sample(cfg.N1, seed=5, rnd=0)
    c32, v32, _ = (N(t) if t is not None else None for t in dev.place_cost(xs, 0, grad=False))
    c64, v64, _, _ = o.place_cost(N(xs), 0, grad=False)
    check_cost("pack tetris8 full batch", c32, c64, v32, v64)


def test_pack_optimize_teacher_forced(sp, orc):
    rng = np.random.default_rng(900)
    prob, pr, _ = synth.config("tetris5", 1)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    x = T(f32(np.concatenate([synth.near_packing(rng, prob, 256), synth.random_placements(rng, prob, 256)])))
    K = pr.k_lin1 + pr.k_quad1
    for k in range(1, K + 1):
        xk = N(x)
        dev.place_optimize(x, k, k + 1)
        x1 = N(x)
        phase, lr = o.schedule(k, pr.k_lin1, pr.eta1, pr.alpha1)
        c, v, g, kink = o.place_cost(xk, phase)
        ref = o.gd_step(xk, g, lr)
        keep = kink >= KINK
        gn = np.linalg.norm(g.reshape(g.shape[0], -1), axis=1)[:, None, None]
        tol = 4 * np.finfo(np.float32).eps * np.abs(xk) + lr * (REL * gn + ABS) + 1e-7
        bad = (np.abs(x1 - ref) > tol) & keep[:, None, None]
        assert not bad.any(), (k, np.argwhere(bad)[:3])
    report("pack teacher forced", steps=K)


def test_pack_place_round_equals_pieces(sp):
    prob, pr, _ = synth.config("tetris5", 0)
    dev = sp.Problem(prob, pr)
    for N_, M_, rnd in [(4096, 1024, 0), (30000, 512, 2)]:
        x, cost, viol, nsat = dev.place_round(N_, M_, seed=3, rnd=rnd)
        xs = dev.sample(N_, 3, rnd)
        c1, _, _ = dev.place_cost(xs, phase=sp.PHASE_LIN, grad=False)
        idx = sp.select_topm_large(c1, M_).long()
        xm = xs[idx].contiguous()
        cq, vq = dev.place_optimize(xm, 1, pr.k_lin1 + pr.k_quad1 + 1)
        ordr, ns = sp.order(cq, vq, pr.sat_eps)
        ordr = ordr.long()
        assert int(N(ns)[0]) == int(N(nsat)[0])
        assert torch.equal(x, xm[ordr]) and torch.equal(cost, cq[ordr]) and torch.equal(viol, vq[ordr])


def test_pack_round_finds_packings(sp, orc):
    """Rounds of the 5-piece workload reach exact packings: the satisfying particles of
    the first rounds that find any are feasible for the FP64 oracle as well."""
    prob, pr, cfg = synth.config("tetris5", 1)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    found = None
    for rnd in range(64):
        x, cost, viol, nsat = dev.place_round(cfg.N1, cfg.M, seed=1, rnd=rnd)
        n = int(N(nsat)[0])
        if n:
            found = (rnd, N(x)[:n], N(viol)[:n])
            break
    assert found is not None
    rnd, xs, vs = found
    _, v64, _, _ = o.place_cost(xs, 1, grad=False)
    report("pack round", round=rnd, satisfying=len(xs), worst_viol=float(v64.max()))
    assert np.all(v64 < 2 * pr.sat_eps)


def test_pack_rejects_stage2(sp):
    prob, pr, cfg = synth.config("tetris5", 0)
    dev = sp.Problem(prob, pr)
    L = sp.load()
    q = torch.zeros(1, 2 * prob.B, 16, 7, device="cuda")
    pose = torch.zeros(1, prob.B, 4, device="cuda")
    with pytest.raises(sp.SpasmError):
        dev.traj_cost(q, pose)
    with pytest.raises(sp.SpasmError):
        dev.ik_lift(pose, seed=0)
    with pytest.raises(sp.SpasmError):
        dev.solve(cfg)
    assert "stage 1 only" in L.spasm_last_error().decode()


def _ragged_pieces(rng, base, B, max_cells=synth.MAX_CELLS):
    """B pieces of 1..max_cells distinct cells each (random lattice shapes, not a tiling)."""
    cells = np.zeros(B, np.int32)
    off = np.zeros((B, synth.MAX_CELLS, 2))
    for b in range(B):
        n = int(rng.integers(1, max_cells + 1))
        pick = rng.choice(16, n, replace=False)
        xy = np.stack([pick % 4, pick // 4], axis=1) * base.h
        off[b, :n] = xy - xy.mean(axis=0)
        cells[b] = n
    region = np.array([0.2, 0.55, -0.2, 0.2])
    return synth.dataclasses.replace(base, block_init=np.zeros((B, 4)), goal=np.tile(base.goal[:1], (B, 1)),
                                     pack_cells=cells, pack_off=off, pack_solution=None, table=region)


@pytest.mark.parametrize("B,N", [(16, 1000), (1, 77), (3, 1021), (2, 500), (8, 300), (15, 257)])
def test_pack_ragged_pieces(sp, orc, B, N):
    """Any pieces of 1..8 cells, up to the 16-piece maximum (128 lanes per particle), on
    particle counts that leave a workgroup partly filled; even piece counts exercise the
    pairs at offset B/2, which only the smaller-numbered piece of each pair takes."""
    rng = np.random.default_rng(300 + B)
    base, pr, _ = synth.config("tetris5", 0)
    prob = _ragged_pieces(rng, base, B)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    x = f32(synth.random_placements(rng, prob, N))
    for phase in (0, 1):
        c32, v32, g32 = (N_(t) for t in dev.place_cost(T(x), phase))
        c64, v64, g64, kink = o.place_cost(x, phase)
        check_cost(f"pack ragged B{B} ph{phase}", c32, c64, v32, v64)
        keep = np.broadcast_to((kink >= KINK)[:, None], g64.shape[:2])
        check_grad(f"pack ragged B{B} ph{phase}", g32, g64, keep)


@pytest.mark.parametrize("steps", [3, 64])
def test_pack_sample_yaw_steps(sp, orc, steps):
    """Yaw on a number of directions that is not a power of two, or the largest allowed:
    the direction index is integer arithmetic on both sides, so it matches exactly."""
    prob, pr, _ = synth.config("tetris5", 2)
    prob = synth.dataclasses.replace(prob, sample_yaw_steps=steps)
    dev = sp.Problem(prob, pr)
    x32 = N_(dev.sample(20000, seed=8, rnd=3))
    x64 = orc.Oracle(prob, pr).sample(20000, 8, 3)
    j32 = np.round((x32[..., 2] + math.pi) / (2 * math.pi / steps)).astype(int)
    j64 = np.round((x64[..., 2] + math.pi) / (2 * math.pi / steps)).astype(int)
    assert np.array_equal(j32, j64) and j64.min() == 0 and j64.max() == steps - 1
    assert np.abs(x32 - x64).max() <= 2e-6


@pytest.mark.parametrize("B", [5, 12])
def test_pack_small_pieces(sp, orc, B):
    """Pieces of at most two cells: four lanes per piece, some of them past every piece's
    last cell."""
    rng = np.random.default_rng(700 + B)
    base, pr, _ = synth.config("tetris5", 0)
    prob = _ragged_pieces(rng, base, B, max_cells=2)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    x = f32(synth.random_placements(rng, prob, 400))
    for phase in (0, 1):
        c32, v32, g32 = (N_(t) for t in dev.place_cost(T(x), phase))
        c64, v64, g64, kink = o.place_cost(x, phase)
        check_cost(f"pack small B{B} ph{phase}", c32, c64, v32, v64)
        keep = np.broadcast_to((kink >= KINK)[:, None], g64.shape[:2])
        check_grad(f"pack small B{B} ph{phase}", g32, g64, keep)
    xs = T(x)
    K = pr.k_lin1 + pr.k_quad1
    cq, vq = dev.place_optimize(xs, 1, K + 1)
    c64, v64, _, _ = o.place_cost(N_(xs), 1, grad=False)
    check_cost(f"pack small B{B} after descent", N_(cq), c64, N_(vq), v64)
