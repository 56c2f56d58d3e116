"""Augmented-Lagrangian outer loop of stage 2 (opt-in, al_every > 0) on the GPU against
the FP64 oracle: the multiplier terms of the cost and gradient, teacher-forced Adam steps
with multiplier updates, and whole solves."""
import numpy as np
import pytest
import torch

from paper_2510_07674_amd import synth
from test_gpu_parity import (ABS, EPS_POS, KINK, REL, N, T, _states, check_cost, check_grad, f32, pose_floor,
                             report, slot_floor)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    from paper_2510_07674_amd import spasm
    spasm.load()
    return spasm


@pytest.mark.parametrize("name,W,P,kind", [("tiny", 16, 32, "lifted"), ("tower4", 32, 4, "lifted"),
                                          ("tower4", 32, 6, "random")])
def test_al_cost_parity(sp, orc, name, W, P, kind):
    rng = np.random.default_rng(400 + P)
    prob, pr, _ = synth.config(name, 5)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    q, pose = _states(kind, prob, pr, orc, rng, P, W)
    q, pose = f32(q), f32(pose)
    lam = f32(rng.normal(0, 2, (P, prob.B, 15)))
    for phase in (0, 1):
        c32, v32, gq32, gp32 = (N(t) for t in dev.traj_cost_al(T(q), T(pose), T(lam), phase))
        c64, v64, gq64, gp64, sk, pk, e = o.traj_cost_al(q, pose, lam, phase)
        # the multiplier terms lambda . e carry the FP32 position error of e times |lambda|
        lam_floor = np.abs(lam).sum(axis=(1, 2)) * EPS_POS
        ec = np.abs(c32 - c64) / (REL * np.abs(c64) + ABS + lam_floor)
        assert np.all(ec <= 1.0), (np.argmax(ec), c32[np.argmax(ec)], c64[np.argmax(ec)])
        assert np.allclose(v32, v64, rtol=REL, atol=10 * ABS)
        keep = sk >= KINK
        fl = slot_floor(pr, q.shape[1], W) + 2 * np.abs(lam).max() * EPS_POS
        check_grad(f"al {name} {kind} ph{phase} q", gq32, gq64, keep, fl)
        pkeep = np.broadcast_to((pk >= KINK)[:, None], gp64.shape[:2])
        check_grad(f"al {name} {kind} ph{phase} pose", gp32, gp64, pkeep, pose_floor(pr) + 2 * np.abs(lam).max() * EPS_POS)
        # zero multipliers give the plain cost bit for bit
        cz, vz, gqz, gpz = dev.traj_cost_al(T(q), T(pose), T(np.zeros_like(lam)), phase)
        c0, v0, gq0, gp0 = dev.traj_cost(T(q), T(pose), phase)
        assert torch.equal(cz, c0) and torch.equal(gqz, gq0) and torch.equal(gpz, gp0)


@pytest.mark.parametrize("name,W,P", [("tiny", 16, 16), ("tower4", 32, 4)])
def test_al_optimize_teacher_forced(sp, orc, name, W, P):
    """Each step from the GPU state: the oracle takes the Adam step with the multiplier
    terms and, every al_every steps, the multiplier step with its own residuals."""
    rng = np.random.default_rng(910)
    prob, pr, cfg = synth.config(name, 7)
    pr = synth.dataclasses.replace(pr, al_every=5, al_rho=1.0)
    dev, o = sp.Problem(prob, pr), orc.Oracle(prob, pr)
    q0, pose0 = _states("lifted", prob, pr, orc, rng, P, W)
    q, pose = T(f32(q0)), T(f32(pose0))
    K = min(cfg.K, 40)
    opt = dev.opt_state(P, W)
    nq = 2 * prob.B * W * 7
    per = nq + 4 * prob.B
    B = prob.B
    w_al = np.array([pr.w_start] * 6 + [pr.w_tie] * 9)
    worst, worst_l = 0.0, 0.0
    for k in range(1, K + 1):
        qk, pk, ok = N(q), N(pose), N(opt)
        lam_k = ok[:, 2 * per:].reshape(P, B, 15)
        dev.traj_optimize(q, pose, opt, k, k + 1, K, want_cost=False)
        q1, p1, o1 = N(q), N(pose), N(opt)
        phase, lr = o.schedule(k, pr.k_lin2(K), pr.eta2, pr.alpha2)
        _, _, gq, gp, sk, pkk, e = o.traj_cost_al(qk, pk, lam_k, phase)
        mq, vq = ok[:, :nq].reshape(qk.shape), ok[:, per:per + nq].reshape(qk.shape)
        mp, vp = ok[:, nq:per].reshape(pk.shape), ok[:, per + nq:2 * per].reshape(pk.shape)
        rq, rp, *_ = o.adam_step(qk, pk, mq, vq, mp, vp, gq, gp, lr, k)
        fl = slot_floor(pr, qk.shape[1], W) + 2 * np.abs(lam_k).max() * EPS_POS
        dg = REL * np.linalg.norm(gq, axis=-1) + fl[None]
        dgs = dg.copy()
        dgs[:, :-1, W - 1] += dg[:, 1:, 0]
        dgs[:, 1:, 0] = dgs[:, :-1, W - 1]
        gsum = gq.copy()
        gsum[:, :-1, W - 1] += gq[:, 1:, 0]
        gsum[:, 1:, 0] = gsum[:, :-1, W - 1]
        vhat = (pr.beta2 * vq + (1 - pr.beta2) * gsum ** 2) / (1 - pr.beta2 ** k)
        ok_c = np.broadcast_to((sk >= KINK)[..., None], qk.shape).copy()
        ok_c[:, :-1, W - 1] &= (sk[:, 1:, 0] >= KINK)[..., None]
        ok_c[:, 1:, 0] &= (sk[:, :-1, W - 1] >= KINK)[..., None]
        tol = 4 * np.finfo(np.float32).eps * np.abs(qk) + 2 * lr * dgs[..., None] / (np.sqrt(vhat) + pr.adam_eps) + 1e-7
        err = np.abs(q1 - rq)
        worst = max(worst, float(np.max(np.where(ok_c, err / tol, 0))))
        assert np.all(err[ok_c] <= tol[ok_c]), (k, np.argwhere(ok_c & (err > tol))[:3])
        # multipliers: unchanged between updates, lam + rho 2w e at every al_every-th step
        lam_1 = o1[:, 2 * per:].reshape(P, B, 15)
        ref = lam_k + (pr.al_rho * 2 * w_al * e if k % pr.al_every == 0 else 0.0)
        tol_l = 4 * np.finfo(np.float32).eps * np.abs(ref) + pr.al_rho * 2 * w_al * 4 * EPS_POS + 1e-6
        worst_l = max(worst_l, float(np.max(np.abs(lam_1 - ref) / tol_l)))
        assert np.all(np.abs(lam_1 - ref) <= tol_l), (k, np.argwhere(np.abs(lam_1 - ref) > tol_l)[:3])
    report(f"al adam {name}", worst_ratio=worst, worst_lambda_ratio=worst_l)


def test_al_solve(sp):
    """Whole solves with the outer loop on: deterministic, ends as the plain solve would
    report them (success by the plain violation), multipliers zeroed at the start of each
    solve (a repeat gives the same result)."""
    for name in ("tiny", "tower4"):
        for seed in synth.certified_seeds(name)[:3]:
            prob, pr, cfg = synth.config(name, seed)
            dev = sp.Problem(prob, synth.dataclasses.replace(pr, al_every=10, al_rho=0.5))
            r1, q1, p1 = dev.solve(cfg)
            r2, q2, p2 = dev.solve(cfg)
            assert torch.equal(q1, q2) and torch.equal(p1, p2) and r1["viol"] == r2["viol"]
            assert r1["success"] == (r1["viol"] < pr.sat_eps)
            t, _, _ = dev.solve_ttfs(cfg, 25, 1)
            report(f"al solve {name} {seed}", success=r1["success"], viol=r1["viol"], ttfs_success=t["success"])
