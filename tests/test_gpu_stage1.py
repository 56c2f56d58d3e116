"""GPU parity of the whole stage 1 (Alg. 1 lines 1-23) and of whole small tower solves
against the FP64 oracle, through the C ABI.

Stage 1, round by round: the samples agree within 1e-6 (24-bit uniforms mapped in each
precision); the M kept samples are exactly the stable sort's first M of the device's own
FP32 scores (the oracle sorts those same keys); the committed round and its satisfying
count equal the oracle's, unless a particle's FP64 violation lies within 1e-5 of the
threshold (FP32 may then decide either way).  Two shortened descent schedules make
satisfying placements rare, so the resampling rounds and the "no round satisfied, lift
the last round anyway" branch run on the device as well.

Whole solves (tower scenes, small sizes): the device's own stage 1, lift and seeding are
taken as the common start, both sides run the K Adam iterations free (FP32 against FP64),
and the per-particle success flags and final violations are compared.
"""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2510_07674_amd import synth
from test_gpu_parity import N, T, f32, report

pytestmark = pytest.mark.gpu

# stage-1 schedules that make satisfying placements rare on the 4-block tower (the oracle
# pins in test_oracle_pins use the same ones): a zero-length linear phase and one
# quadratic step (no round satisfies), or a short linear phase (the first round of some
# scenes has no satisfying particle, a later one does)
NO_SAT = dict(k_lin1=1, k_quad1=1, alpha1=0.5)
RARE_SAT = dict(k_lin1=2, k_quad1=1, alpha1=0.1)
NEAR = 1e-5   # FP64 violations this close to the threshold may be decided either way in FP32


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    from paper_2510_07674_amd import spasm
    spasm.load()
    return spasm


def _problem(sched, k):
    prob, pr, _ = synth.config("tower4", synth.certified_seeds("tower4")[k])
    if sched:
        pr = dataclasses.replace(pr, **sched)
    return prob, pr


def test_sample_placements_is_top_m_of_scores(sp, orc):
    """Alg. 1 lines 1-4: the kept placements are the stable sort's first M of the device's
    own linear scores (compared bit for bit, the oracle sorting the same FP32 keys), and
    those scores match the oracle's FP64 scores of the same samples."""
    for name, N_, M_, rnd in [("tower4", 4096, 1024, 0), ("tower10", 16384, 2048, 1), ("tower4", 40000, 512, 2),
                              ("tower4", 100, 100, 0), ("tetris5", 3000, 7, 3)]:
        prob, pr, _ = synth.config(name, synth.instance_seeds(name)[0])
        dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
        x, c, v = (N(t) for t in dev.sample_placements(N_, M_, seed=11, rnd=rnd))
        xs = dev.sample(N_, 11, rnd)
        c_all, v_all, _ = dev.place_cost(xs, phase=sp.PHASE_LIN, grad=False)
        c_all, v_all, xs = N(c_all), N(v_all), N(xs)
        idx = orc.Oracle.argsort(c_all)[:M_]
        assert np.array_equal(x, xs[idx]) and np.array_equal(c, c_all[idx]) and np.array_equal(v, v_all[idx])
        assert np.abs(xs - o.sample(N_, 11, rnd)).max() <= 1e-6
        pick = idx[:64]
        c64, v64, _, _ = o.place_cost(f32(xs[pick]), 0, grad=False)
        assert np.all(np.abs(c[:64] - c64) <= 1e-4 * np.abs(c64) + 1e-6), name
        report(f"sample_placements {name}", N=N_, M=M_, best=float(c[0]))


def _near(v64, eps):
    return bool(np.any(np.abs(v64 - eps) < NEAR))


@pytest.mark.parametrize("sched", [None, RARE_SAT, NO_SAT], ids=["default", "rare", "none"])
def test_stage1_rounds_vs_oracle(sp, orc, sched):
    """The device's whole stage 1 equals its single rounds composed as Alg. 1 composes them,
    and takes the same rounds and satisfying counts as the FP64 oracle's stage 1."""
    resampled = exhausted = 0
    for k in range(8):
        prob, pr = _problem(sched, k)
        dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
        N_, M_, seed = (64, 8, 3) if k % 2 == 0 else (256, 16, 5)
        pose, cost, viol, info = dev.stage1(N_, M_, seed)
        pose, cost, viol, info = N(pose), N(cost), N(viol), N(info).astype(np.int64)
        # device rounds, one at a time
        want = None
        for r in range(pr.retries + 1):
            x_r, c_r, v_r, ns_r = (N(t) for t in dev.place_round(N_, M_, seed=seed, rnd=r))
            if int(ns_r[0]) > 0 or r == pr.retries:
                want = (r, x_r, c_r, v_r, int(ns_r[0]))
                break
        r, x_r, c_r, v_r, ns = want
        assert int(info[1]) == r + 1 and int(info[0]) == ns, (k, info, r, ns)
        assert np.array_equal(pose[..., [0, 1, 3]], x_r) and np.array_equal(cost, c_r) and np.array_equal(viol, v_r)
        assert np.allclose(pose[..., 2], (np.arange(prob.B) + 0.5)[None] * prob.h, rtol=0, atol=1e-7)
        # the oracle's rounds: same stopping round and satisfying count
        ok, ns64 = True, -1
        for ro in range(pr.retries + 1):
            _, c64, v64 = o.stage1(N_, M_, seed, ro)
            if _near(v64, pr.sat_eps):
                ok = False
                break
            _, ns64 = o.order(c64, v64)
            if ns64 > 0:
                break
        rounds64 = ro + 1
        report(f"stage1 {sched and sched['k_lin1']} scene {k}", rounds=r + 1, nsat=ns, oracle_rounds=rounds64,
               oracle_nsat=ns64 if ok else -1)
        if ok:
            assert rounds64 == r + 1 and ns64 == ns, (k, rounds64, ns64)
        resampled += r > 0
        exhausted += ns == 0
    if sched is RARE_SAT:
        assert resampled > 0   # some scene needed a second round
    if sched is NO_SAT:
        assert exhausted == 8  # every scene lifted its last round's particles


@pytest.mark.parametrize("k", range(8))
def test_tower_solve_vs_oracle(sp, orc, k):
    """A small tower solve: the device pipeline equals its pieces bit for bit, and from the
    device's stage-1, lift and seeding state the FP64 oracle's K Adam iterations reach the
    same success (any particle) and per-particle success flags for at least 90 % of the
    particles (those within 1e-5 of the threshold aside; 97-100 % measured), and where
    both stay infeasible violations within a factor 2 for at least 80 % of them."""
    prob, pr = _problem(None, k)
    cfg = synth.SolveConfig(N1=512, M=32, W=16, K=120, seed=7)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    res, bq, bp = dev.solve(cfg)
    pose, _, _, info = dev.stage1(cfg.N1, cfg.M, cfg.seed)
    qg, qp = dev.ik_lift(pose, cfg.seed)
    q = dev.traj_init(qg, qp, cfg.W, cfg.seed, pose)
    q0, p0 = N(q), N(pose)
    opt = dev.opt_state(cfg.M, cfg.W)
    c32, v32 = dev.traj_optimize(q, pose, opt, 1, cfg.K + 1, cfg.K)
    c32, v32 = N(c32), N(v32)
    ordr, ns = sp.order(T(c32), T(v32), pr.sat_eps)
    best = int(N(ordr)[0])
    assert res["rounds"] == int(N(info)[1]) and res["best"] == best and res["viol"] == np.float32(v32[best])
    assert torch.equal(bq, q[best]) and torch.equal(bp, pose[best])
    # FP64 from the same start
    q64, p64 = o.stage2(q0, p0, cfg.K)
    c64, v64 = o.traj_cost(q64, p64, 1, grad=False)[:2]
    s32, s64 = v32 < pr.sat_eps, v64 < pr.sat_eps
    decided = np.abs(v64 - pr.sat_eps) >= NEAR
    agree = float(np.mean((s32 == s64)[decided]))
    report(f"tower solve {k}", gpu_success=int(res["success"]), gpu_nsat=int(s32.sum()), oracle_nsat=int(s64.sum()),
           agree=agree, gpu_best_v=float(v32.min()), oracle_best_v=float(v64.min()), rounds=res["rounds"])
    assert (s32.any() == s64.any()) or not decided.all()
    assert agree >= 0.9
    # where both runs stay infeasible their violations are of the same size (within 2x):
    # the two precisions stall in the same contact
    both = (v32 >= pr.sat_eps) & (v64 >= pr.sat_eps)
    ratio = np.abs(np.log(v32[both] / v64[both])) if both.any() else np.zeros(1)
    assert np.mean(ratio <= np.log(2.0)) >= 0.8, np.sort(ratio)[-4:]


@pytest.mark.parametrize("k", range(3))
def test_tower10_solve_vs_oracle(sp, orc, k):
    """A small 10-block tower solve (80 boxes, 20 segments of 32 waypoints): the device
    pipeline equals its pieces bit for bit, and from the device's stage-1, lift and
    seeding state the FP64 oracle's K Adam iterations end in the same success flags (those
    within 1e-5 of the threshold aside) and, where both stay infeasible, violations within
    a factor 2 for at least 80 % of the particles."""
    prob, pr, _ = synth.config("tower10", synth.certified_seeds("tower10")[k])
    cfg = synth.SolveConfig(N1=2048, M=32, W=32, K=300, seed=11)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    res, bq, bp = dev.solve(cfg)
    pose, _, _, info = dev.stage1(cfg.N1, cfg.M, cfg.seed)
    qg, qp = dev.ik_lift(pose, cfg.seed)
    q = dev.traj_init(qg, qp, cfg.W, cfg.seed, pose)
    q0, p0 = N(q), N(pose)
    opt = dev.opt_state(cfg.M, cfg.W)
    c32, v32 = dev.traj_optimize(q, pose, opt, 1, cfg.K + 1, cfg.K)
    c32, v32 = N(c32), N(v32)
    ordr, _ = sp.order(T(c32), T(v32), pr.sat_eps)
    best = int(N(ordr)[0])
    assert res["rounds"] == int(N(info)[1]) and res["best"] == best and res["viol"] == np.float32(v32[best])
    assert torch.equal(bq, q[best]) and torch.equal(bp, pose[best])
    q64, p64 = o.stage2(q0, p0, cfg.K)
    c64, v64 = o.traj_cost(q64, p64, 1, grad=False)[:2]
    s32, s64 = v32 < pr.sat_eps, v64 < pr.sat_eps
    decided = np.abs(v64 - pr.sat_eps) >= NEAR
    both = (v32 >= pr.sat_eps) & (v64 >= pr.sat_eps)
    ratio = np.abs(np.log(v32[both] / v64[both])) if both.any() else np.zeros(1)
    report(f"tower10 solve {k}", gpu_nsat=int(s32.sum()), oracle_nsat=int(s64.sum()),
           flags_agree=float(np.mean((s32 == s64)[decided])), within2=float(np.mean(ratio <= np.log(2.0))),
           gpu_best_v=float(v32.min()), oracle_best_v=float(v64.min()), max_log_ratio=float(ratio.max()))
    assert np.all((s32 == s64)[decided])
    assert np.mean(ratio <= np.log(2.0)) >= 0.8, np.sort(ratio)[-4:]
