"""FP64 CPU oracle of the SPaSM hot path -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper over ``liboracle.so`` (plain C, FP64, OpenMP over particles).  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It shares no code with the HIP library; both read the same problem
descriptions produced by ``paper_2510_07674_amd.synth``.

The pipeline glue (``solve``) follows Alg. 1 and Sec. III-B of the paper: stage 1
(sample, score, top-M, linear then quadratic descent, satisfying-first order, bounded
resampling), lift by IK, trajectory seeding, stage-2 Adam descent, best particle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

LIN, QUAD = 0, 1
MODE_TOWER, MODE_FIXED, MODE_PACK, MODE_P2P = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile liboracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-shared", "-fPIC",
                               os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Prob(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int), ("O", ctypes.c_int), ("B", ctypes.c_int), ("mode", ctypes.c_int),
                ("dh", ctypes.c_void_p), ("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p),
                ("tool_d", ctypes.c_double), ("q_home", ctypes.c_void_p),
                ("sph_link", ctypes.c_void_p), ("sph_c", ctypes.c_void_p), ("sph_r", ctypes.c_void_p),
                ("boxes", ctypes.c_void_p), ("h", ctypes.c_double), ("block_margin", ctypes.c_double),
                ("block_init", ctypes.c_void_p), ("goal", ctypes.c_void_p), ("grasp", ctypes.c_void_p),
                ("table", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("pack_cells", ctypes.c_void_p), ("pack_off", ctypes.c_void_p),
                ("sample_yaw_steps", ctypes.c_int), ("p2p_goal", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_Prob)
        vp, i, d, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
        L.or_philox4x64_10.argtypes = [vp, vp, vp]
        L.or_fk.argtypes = [P, vp, vp]
        L.or_box_sdf.argtypes = [vp, vp, vp]
        L.or_box_sdf.restype = d
        L.or_obb_sdf.argtypes = [vp, vp, d, vp, vp]
        L.or_obb_sdf.restype = d
        L.or_square_pen.argtypes = [vp, d, vp, d, d, vp]
        L.or_square_pen.restype = d
        L.or_place_cost.argtypes = [P, i, i, i, vp, vp, vp, vp, vp]
        L.or_traj_cost.argtypes = [P, i, i, i, vp, vp, vp, vp, vp, vp, vp, vp]
        L.or_traj_cost_al.argtypes = [P, i, i, i, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.or_traj_residuals.argtypes = [P, i, i, vp, vp, vp]
        L.or_traj_slot_residuals.argtypes = [P, i, i, vp, vp, vp]
        L.or_box_clearance.argtypes = [P, i, vp, vp, i, vp, vp]
        L.or_al_update.argtypes = [P, i, vp, d, vp]
        L.or_stage2_al.argtypes = [P, i, i, i, i, d, d, d, d, d, i, d, vp, vp, vp]
        L.or_schedule.argtypes = [i, i, d, d, vp, vp]
        L.or_gd_step.argtypes = [P, i, vp, vp, d]
        L.or_traj_adam_step.argtypes = [P, i, i, vp, vp, vp, vp, vp, vp, vp, vp, d, i, d, d, d]
        L.or_sample.argtypes = [P, i, u64, i, vp]
        L.or_argsort.argtypes = [i, vp, vp]
        L.or_order.argtypes = [i, vp, vp, d, vp, vp]
        L.or_ik_iterate.argtypes = [P, i, vp, vp, i, d]
        L.or_ik_lift.argtypes = [P, i, vp, u64, i, d, d, i, vp, vp]
        L.or_ik_error.argtypes = [P, i, vp, vp]
        L.or_ik_error.restype = d
        L.or_arm_clutter.argtypes = [P, vp, vp, i, i]
        L.or_arm_clutter.restype = d
        L.or_traj_init.argtypes = [P, i, i, vp, vp, vp, u64, d, i, vp]
        L.or_stage1.argtypes = [P, i, i, u64, i, i, i, d, d, vp, vp, vp]
        L.or_stage2.argtypes = [P, i, i, i, i, d, d, d, d, d, vp, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Binds one problem (synth.Problem) and its parameters (synth.Params)."""

    def __init__(self, prob, params):
        self.prob, self.params = prob, params
        self._keep = {
            "dh": _f64(prob.dh), "lo": _f64(prob.lo), "hi": _f64(prob.hi), "q_home": _f64(prob.q_home),
            "sph_link": np.ascontiguousarray(prob.sph_link, dtype=np.int32),
            "sph_c": _f64(prob.sph_c), "sph_r": _f64(prob.sph_r),
            "boxes": _f64(prob.boxes).reshape(-1, 6) if prob.O else np.zeros((1, 6)),
            "block_init": _f64(prob.block_init), "goal": _f64(prob.goal), "grasp": _f64(prob.grasp),
            "table": _f64(prob.table), "w": _f64(params.weights()),
            "pack_cells": (np.ascontiguousarray(prob.pack_cells, dtype=np.int32)
                           if getattr(prob, "pack_cells", None) is not None else None),
            "pack_off": (_f64(prob.pack_off) if getattr(prob, "pack_off", None) is not None else None),
            "p2p_goal": (_f64(prob.p2p_goal) if getattr(prob, "p2p_goal", None) is not None else None),
        }
        k = self._keep
        self.c = _Prob(prob.S, prob.O, prob.B, prob.mode, _ptr(k["dh"]).value, _ptr(k["lo"]).value,
                       _ptr(k["hi"]).value, prob.tool_d, _ptr(k["q_home"]).value,
                       _ptr(k["sph_link"]).value, _ptr(k["sph_c"]).value, _ptr(k["sph_r"]).value,
                       _ptr(k["boxes"]).value, prob.h, prob.block_margin, _ptr(k["block_init"]).value,
                       _ptr(k["goal"]).value, _ptr(k["grasp"]).value, _ptr(k["table"]).value,
                       _ptr(k["w"]).value,
                       _ptr(k["pack_cells"]).value if k["pack_cells"] is not None else None,
                       _ptr(k["pack_off"]).value if k["pack_off"] is not None else None,
                       int(getattr(prob, "sample_yaw_steps", 0)),
                       _ptr(k["p2p_goal"]).value if k["p2p_goal"] is not None else None)
        self.ref = ctypes.byref(self.c)

    # -- geometry -------------------------------------------------------------------------
    def fk(self, q) -> np.ndarray:
        q = _f64(q)
        out = np.zeros((9, 12))
        lib().or_fk(self.ref, _ptr(q), _ptr(out))
        return out

    # -- costs ----------------------------------------------------------------------------
    @staticmethod
    def square_pen(ca, tha, cb, thb, s):
        """Penetration depth of two squares of half edge s (separating axis theorem) and its
        gradient d/d(ca_x, ca_y, tha, cb_x, cb_y, thb), plus the kink margin."""
        ca, cb = _f64(ca), _f64(cb)
        g = np.zeros(7)
        pen = lib().or_square_pen(_ptr(ca), float(tha), _ptr(cb), float(thb), float(s), _ptr(g))
        return pen, g[:6], g[6]

    def place_cost(self, x, phase=LIN, grad=True, dim=None):
        x = _f64(x)
        N, B, D = x.shape
        dim = D if dim is None else dim
        cost, viol, kink = np.zeros(N), np.zeros(N), np.zeros(N)
        g = np.zeros_like(x) if grad else None
        lib().or_place_cost(self.ref, dim, phase, N, _ptr(x), _ptr(cost), _ptr(viol),
                            _ptr(g) if grad else None, _ptr(kink))
        return cost, viol, g, kink

    def traj_cost(self, q, pose, phase=LIN, grad=True):
        q, pose = _f64(q), _f64(pose)
        P, NS, W, _ = q.shape
        cost, viol, pk = np.zeros(P), np.zeros(P), np.zeros(P)
        sk = np.zeros((P, NS, W))
        gq = np.zeros_like(q) if grad else None
        gp = np.zeros_like(pose) if grad else None
        lib().or_traj_cost(self.ref, phase, P, W, _ptr(q), _ptr(pose), _ptr(cost), _ptr(viol),
                           _ptr(gq) if grad else None, _ptr(gp) if grad else None, _ptr(sk), _ptr(pk))
        return cost, viol, gq, gp, sk, pk

    RESIDUALS = ("arm_box", "arm_block", "held_box", "held_block", "grasp", "tie", "limit", "place")

    def traj_residuals(self, q, pose):
        """Per particle, the largest residual of each kind in RESIDUALS (their maximum is the
        violation): [P, 8]."""
        q, pose = _f64(q), _f64(pose)
        out = np.zeros((q.shape[0], len(self.RESIDUALS)))
        lib().or_traj_residuals(self.ref, q.shape[0], q.shape[2], _ptr(q), _ptr(pose), _ptr(out))
        return out

    def traj_slot_residuals(self, q, pose):
        """The breakdown per waypoint slot: [P, NS, W, 8] (placement entry zero)."""
        q, pose = _f64(q), _f64(pose)
        out = np.zeros(q.shape[:3] + (len(self.RESIDUALS),))
        lib().or_traj_slot_residuals(self.ref, q.shape[0], q.shape[2], _ptr(q), _ptr(pose), _ptr(out))
        return out

    def box_clearance(self, q, pose, boxes):
        """Smallest sdf - r of one plan (q [NS, W, 7], pose [B, 4]) against each box of
        boxes [n, 6]: robot spheres at every slot, the held block inside transfers, every
        block at its initial pose and at its placement."""
        q, pose, boxes = _f64(q), _f64(pose), _f64(boxes).reshape(-1, 6)
        out = np.zeros(boxes.shape[0])
        lib().or_box_clearance(self.ref, q.shape[1], _ptr(q), _ptr(pose), boxes.shape[0], _ptr(boxes), _ptr(out))
        return out

    def traj_cost_al(self, q, pose, lam, phase=LIN, grad=True):
        """Stage-2 cost with the multiplier terms lambda . e (lam [P, B, 15]); also returns
        the equality residuals e [P, B, 15] (grasp rp, rz; tie rp, rx, rz per block)."""
        q, pose, lam = _f64(q), _f64(pose), _f64(lam)
        P, NS, W, _ = q.shape
        cost, viol, pk = np.zeros(P), np.zeros(P), np.zeros(P)
        sk = np.zeros((P, NS, W))
        e = np.zeros((P, self.prob.B, 15))
        gq = np.zeros_like(q) if grad else None
        gp = np.zeros_like(pose) if grad else None
        lib().or_traj_cost_al(self.ref, phase, P, W, _ptr(q), _ptr(pose), _ptr(lam), _ptr(e), _ptr(cost),
                              _ptr(viol), _ptr(gq) if grad else None, _ptr(gp) if grad else None, _ptr(sk),
                              _ptr(pk))
        return cost, viol, gq, gp, sk, pk, e

    def al_update(self, e, lam, rho):
        lam = _f64(lam).copy()
        lib().or_al_update(self.ref, lam.shape[0], _ptr(_f64(e)), rho, _ptr(lam))
        return lam

    # -- updates --------------------------------------------------------------------------
    @staticmethod
    def schedule(k, k_lin, eta, alpha):
        ph, lr = ctypes.c_int(), ctypes.c_double()
        lib().or_schedule(k, k_lin, eta, alpha, ctypes.byref(ph), ctypes.byref(lr))
        return ph.value, lr.value

    def gd_step(self, x, g, lr):
        x = _f64(x).copy()
        lib().or_gd_step(self.ref, x.shape[0], _ptr(x), _ptr(_f64(g)), lr)
        return x

    def adam_step(self, q, pose, mq, vq, mp, vp, gq, gp, lr, t):
        q, pose, mq, vq, mp, vp = (_f64(a).copy() for a in (q, pose, mq, vq, mp, vp))
        pr = self.params
        lib().or_traj_adam_step(self.ref, q.shape[0], q.shape[2], _ptr(q), _ptr(pose), _ptr(mq), _ptr(vq),
                                _ptr(mp), _ptr(vp), _ptr(_f64(gq)), _ptr(_f64(gp)), lr, t,
                                pr.beta1, pr.beta2, pr.adam_eps)
        return q, pose, mq, vq, mp, vp

    # -- sampling / selection ---------------------------------------------------------------
    def sample(self, N, seed, rnd=0):
        x = np.zeros((N, self.prob.B, 3))
        lib().or_sample(self.ref, N, seed, rnd, _ptr(x))
        return x

    @staticmethod
    def argsort(key):
        key = _f64(key)
        idx = np.zeros(key.shape[0], dtype=np.int32)
        lib().or_argsort(key.shape[0], _ptr(key), _ptr(idx))
        return idx

    def order(self, cost, viol):
        cost, viol = _f64(cost), _f64(viol)
        order = np.zeros(cost.shape[0], dtype=np.int32)
        ns = np.zeros(1, dtype=np.int32)
        lib().or_order(cost.shape[0], _ptr(cost), _ptr(viol), self.params.sat_eps, _ptr(order), _ptr(ns))
        return order, int(ns[0])

    # -- lift / init --------------------------------------------------------------------------
    def ik_iterate(self, kind, target, q, iters):
        q = _f64(q).copy()
        lib().or_ik_iterate(self.ref, kind, _ptr(_f64(target)), _ptr(q), iters, self.params.ik_lambda)
        return q

    def ik_error(self, kind, target, q):
        """|e| of the IK iteration at q (position and orientation error of the block frame)."""
        return lib().or_ik_error(self.ref, kind, _ptr(_f64(target)), _ptr(_f64(q)))

    def arm_clutter(self, q, pose, b, kind):
        """Arm clutter score at q for block b: sum over robot spheres of max(0, r - sdf)
        against the boxes and the blocks visible in situation kind (0 grasp, 1 place,
        2 transit interior, 3 transfer interior); pose [B, 4] the particle's placements."""
        return lib().or_arm_clutter(self.ref, _ptr(_f64(q)), _ptr(_f64(pose)), b, kind)

    def ik_lift(self, pose, seed, iters=None):
        pose = _f64(pose)
        P, B = pose.shape[:2]
        qg, qp = np.zeros((P, B, 7)), np.zeros((P, B, 7))
        pr = self.params
        lib().or_ik_lift(self.ref, P, _ptr(pose), seed, pr.ik_iters if iters is None else iters,
                         pr.ik_lambda, pr.ik_noise, pr.ik_restarts, _ptr(qg), _ptr(qp))
        return qg, qp

    def traj_init(self, qg, qp, W, seed, pose):
        """Seeds; pose [P, B, 4] the placements (the intermediate-waypoint choice sees the
        blocks at them)."""
        qg, qp, pose = _f64(qg), _f64(qp), _f64(pose)
        P, B = qg.shape[:2]
        # a point-to-point problem has one motion (start to goal); qg, qp and pose unused
        q = np.zeros((P, 1 if self.prob.mode == MODE_P2P else 2 * B, W, 7))
        lib().or_traj_init(self.ref, P, W, _ptr(qg), _ptr(qp), _ptr(pose), seed, self.params.mid_noise,
                           self.params.mid_candidates, _ptr(q))
        return q

    def p2p_init(self, P, W, seed):
        """Seeds of a point-to-point problem: [P, 1, W, 7] from q_home to p2p_goal."""
        z = np.zeros((P, self.prob.B, 7))
        return self.traj_init(z, z, W, seed, np.zeros((P, self.prob.B, 4)))

    # -- drivers ---------------------------------------------------------------------------
    def stage1(self, N, M, seed, rnd=0):
        pr = self.params
        x = np.zeros((M, self.prob.B, 3))
        c, v = np.zeros(M), np.zeros(M)
        lib().or_stage1(self.ref, N, M, seed, rnd, pr.k_lin1, pr.k_quad1, pr.eta1, pr.alpha1,
                        _ptr(x), _ptr(c), _ptr(v))
        return x, c, v

    def stage2(self, q, pose, K, lam=None):
        """K Adam iterations; with params.al_every > 0 the augmented-Lagrangian multipliers
        lam [P, B, 15] (zeros when None) are updated in place and returned too."""
        q, pose = _f64(q).copy(), _f64(pose).copy()
        pr = self.params
        every = int(getattr(pr, "al_every", 0))
        if every > 0:
            lam = np.zeros((q.shape[0], self.prob.B, 15)) if lam is None else _f64(lam).copy()
        lib().or_stage2_al(self.ref, q.shape[0], q.shape[2], K, pr.k_lin2(K), pr.eta2, pr.alpha2,
                           pr.beta1, pr.beta2, pr.adam_eps, every, float(getattr(pr, "al_rho", 0.0)), _ptr(q),
                           _ptr(pose), _ptr(lam) if every > 0 else None)
        return (q, pose, lam) if every > 0 else (q, pose)

    def initial_poses(self, x):
        """Stage-1 placements (x, y, yaw) -> stage-2 pose variables (x, y, z*, yaw)."""
        prob = self.prob
        M, B = x.shape[:2]
        pose = np.zeros((M, B, 4))
        pose[..., 0] = x[..., 0]
        pose[..., 1] = x[..., 1]
        pose[..., 2] = (np.arange(B) + 0.5)[None, :] * prob.h
        pose[..., 3] = x[..., 2]
        return pose

    def solve(self, cfg):
        """Whole method in FP64: returns dict(success, viol, cost, q, pose, order info)."""
        prob, pr = self.prob, self.params
        if cfg.N1 > 0:
            # Alg. 1: resample while no particle satisfies, at most `retries` more rounds;
            # the last round's particles are lifted when none ever does
            for rnd in range(pr.retries + 1):
                x, c1, v1 = self.stage1(cfg.N1, cfg.M, cfg.seed, rnd)
                order, nsat = self.order(c1, v1)
                if nsat > 0:
                    break
            rounds = rnd + 1
            pose = self.initial_poses(x[order])
        else:
            nsat, rounds = -1, 0
            pose = np.repeat(_f64(prob.goal)[None], cfg.M, axis=0)
        pose0 = pose
        qg, qp = self.ik_lift(pose, cfg.seed)
        q = self.traj_init(qg, qp, cfg.W, cfg.seed, pose)
        q, pose = self.stage2(q, pose, cfg.K)
        cost, viol = self.traj_cost(q, pose, phase=QUAD, grad=False)[:2]
        order2, nsat2 = self.order(cost, viol)
        best = int(order2[0])
        return {"success": nsat2 > 0, "viol": viol, "cost": cost, "best": best, "n_sat": nsat2,
                "stage1_sat": nsat, "rounds": rounds, "pose0": pose0, "q": q, "pose": pose}
