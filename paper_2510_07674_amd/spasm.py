"""Thin Python binding of libspasm.so (argument marshalling only).

Every step of the method runs in the HIP kernels behind the C ABI declared in
include/spasm.h; this module converts problem descriptions to the C structs, checks
tensor shapes/devices, and passes device pointers plus the current torch stream.
There is no CPU fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspasm.so")

STAGE_PLACE, STAGE_TRAJ = 1, 2
MODE_TOWER, MODE_FIXED, MODE_PACK, MODE_P2P = 0, 1, 2, 3
PHASE_LIN, PHASE_QUAD = 0, 1

c_d, c_i32, c_u64, c_vp = ctypes.c_double, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p


class ChainDesc(ctypes.Structure):
    _fields_ = [("dh", c_d * 21), ("lo", c_d * 7), ("hi", c_d * 7), ("tool_d", c_d), ("q_home", c_d * 7)]


class SkeletonDesc(ctypes.Structure):
    _fields_ = [("n_blocks", c_i32), ("mode", c_i32), ("block_edge", c_d), ("block_margin", c_d),
                ("block_init", c_vp), ("goal", c_vp), ("grasp", c_d * 12), ("region", c_d * 4),
                ("pack_cells", c_vp), ("pack_off", c_vp), ("sample_yaw_steps", c_i32), ("p2p_goal", c_vp)]


class ParamsDesc(ctypes.Structure):
    _fields_ = [("w", c_d * 9), ("k_lin1", c_i32), ("k_quad1", c_i32), ("eta1", c_d), ("alpha1", c_d),
                ("lin_frac2", c_d), ("eta2", c_d), ("alpha2", c_d), ("beta1", c_d), ("beta2", c_d),
                ("adam_eps", c_d), ("ik_iters", c_i32), ("ik_restarts", c_i32), ("mid_candidates", c_i32), ("ik_lambda", c_d), ("ik_noise", c_d),
                ("mid_noise", c_d), ("sat_eps", c_d), ("retries", c_i32), ("al_every", c_i32), ("al_rho", c_d)]


class SolveConfigDesc(ctypes.Structure):
    _fields_ = [("N1", c_i32), ("M", c_i32), ("W", c_i32), ("K", c_i32), ("seed", c_u64)]


class ResultDesc(ctypes.Structure):
    _fields_ = [("success", c_i32), ("n_sat", c_i32), ("stage1_sat", c_i32), ("rounds", c_i32), ("best", c_i32),
                ("viol", ctypes.c_float), ("cost", ctypes.c_float), ("length", ctypes.c_float),
                ("stage1_ms", ctypes.c_float), ("stage2_ms", ctypes.c_float), ("total_ms", ctypes.c_float),
                ("opt_ms", ctypes.c_float)]


class CompletionDesc(ctypes.Structure):
    _fields_ = [("req_id", c_u64), ("status", c_i32), ("steps", c_i32), ("result", ResultDesc)]


SYMBOLS = {
    "spasm_problem_create": ([ctypes.POINTER(ChainDesc), c_i32, c_vp, c_vp, c_vp, c_i32, c_vp,
                              ctypes.POINTER(SkeletonDesc), ctypes.POINTER(ParamsDesc), ctypes.POINTER(c_vp)], c_i32),
    "spasm_problem_destroy": ([c_vp], None),
    "spasm_problem_blocks": ([c_vp], c_i32),
    "spasm_sample": ([c_vp, c_i32, c_u64, c_i32, c_vp, c_vp], c_i32),
    "spasm_cost_grad": ([c_vp, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp], c_i32),
    "spasm_cost_adjoint": ([c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp], c_i32),
    "spasm_cost_grad_al": ([c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp], c_i32),
    "spasm_optimize": ([c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp], c_i32),
    "spasm_select_topm": ([c_i32, c_vp, c_i32, c_vp, c_vp], c_i32),
    "spasm_order": ([c_i32, c_vp, c_vp, ctypes.c_float, c_vp, c_vp, c_vp], c_i32),
    "spasm_select_topm_workspace": ([c_i32, c_i32], ctypes.c_size_t),
    "spasm_select_topm_large": ([c_i32, c_vp, c_i32, c_vp, c_vp, ctypes.c_size_t, c_vp], c_i32),
    "spasm_select_topm_static_bytes": ([], ctypes.c_size_t),
    "spasm_select_topm_static": ([c_i32, c_vp, c_i32, c_vp, c_vp], c_i32),
    "spasm_place_workspace": ([c_vp, c_i32, c_i32], ctypes.c_size_t),
    "spasm_place_round": ([c_vp, c_i32, c_i32, c_u64, c_i32, c_vp, ctypes.c_size_t, c_vp, c_vp, c_vp, c_vp, c_vp],
                          c_i32),
    "spasm_sample_placements_workspace": ([c_vp, c_i32, c_i32], ctypes.c_size_t),
    "spasm_sample_placements": ([c_vp, c_i32, c_i32, c_u64, c_i32, c_vp, ctypes.c_size_t, c_vp, c_vp, c_vp, c_vp],
                                c_i32),
    "spasm_stage1_workspace": ([c_vp, c_i32, c_i32], ctypes.c_size_t),
    "spasm_stage1": ([c_vp, c_i32, c_i32, c_u64, c_vp, ctypes.c_size_t, c_vp, c_vp, c_vp, c_vp, c_vp], c_i32),
    "spasm_ik_iterate": ([c_vp, c_i32, c_i32, c_vp, c_vp, c_i32, c_vp], c_i32),
    "spasm_ik_lift": ([c_vp, c_i32, c_vp, c_u64, c_i32, c_vp, c_vp, c_vp], c_i32),
    "spasm_traj_init": ([c_vp, c_i32, c_i32, c_vp, c_vp, c_vp, c_u64, c_vp, c_vp], c_i32),
    "spasm_solve_workspace": ([c_vp, ctypes.POINTER(SolveConfigDesc)], ctypes.c_size_t),
    "spasm_solve_footprint": ([c_vp, ctypes.POINTER(SolveConfigDesc)], ctypes.c_size_t),
    "spasm_solve_ttfs_workspace": ([c_vp, ctypes.POINTER(SolveConfigDesc)], ctypes.c_size_t),
    "spasm_solve_ttfs": ([c_vp, ctypes.POINTER(SolveConfigDesc), c_i32, c_i32, c_vp, ctypes.c_size_t, c_vp, c_vp,
                          ctypes.POINTER(ResultDesc), ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), c_vp], c_i32),
    "spasm_solve": ([c_vp, ctypes.POINTER(SolveConfigDesc), c_vp, ctypes.c_size_t, c_vp, c_vp,
                     ctypes.POINTER(ResultDesc), c_vp], c_i32),
    "spasm_server_footprint": ([c_vp, ctypes.POINTER(SolveConfigDesc)], ctypes.c_size_t),
    "spasm_server_create": ([ctypes.c_size_t, c_i32, c_i32, ctypes.POINTER(c_vp)], c_i32),
    "spasm_server_submit": ([c_vp, c_vp, ctypes.POINTER(SolveConfigDesc), c_u64, c_vp, c_vp], c_i32),
    "spasm_server_step": ([c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)], c_i32),
    "spasm_server_poll": ([c_vp, ctypes.POINTER(CompletionDesc), c_i32, ctypes.POINTER(c_i32)], c_i32),
    "spasm_server_destroy": ([c_vp], None),
    "spasm_last_error": ([], ctypes.c_char_p),
}

_lib = None


class SpasmError(RuntimeError):
    pass


def load():
    """Load libspasm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SpasmError(f"{LIB_PATH} is missing: build it with paper_2510_07674_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SYMBOLS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SpasmError(f"spasm error {rc}: {load().spasm_last_error().decode()}")


def _stream():
    return c_vp(torch.cuda.current_stream().cuda_stream)


def _dev(t, shape=None, dtype=torch.float32, name="tensor"):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise SpasmError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise SpasmError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return c_vp(t.data_ptr())


def _empty(*shape, dtype=torch.float32):
    return torch.empty(shape, dtype=dtype, device="cuda")


def chain_desc(prob) -> ChainDesc:
    c = ChainDesc()
    c.dh[:] = [float(v) for v in np.asarray(prob.dh, dtype=np.float64).ravel()]
    c.lo[:] = [float(v) for v in prob.lo]
    c.hi[:] = [float(v) for v in prob.hi]
    c.tool_d = float(prob.tool_d)
    c.q_home[:] = [float(v) for v in prob.q_home]
    return c


def params_desc(pr) -> ParamsDesc:
    p = ParamsDesc()
    p.w[:] = [float(v) for v in pr.weights()]
    for name in ("k_lin1", "k_quad1", "ik_iters", "ik_restarts", "mid_candidates", "retries"):
        setattr(p, name, int(getattr(pr, name)))
    p.al_every = int(getattr(pr, "al_every", 0))
    p.al_rho = float(getattr(pr, "al_rho", 1.0))
    for name in ("eta1", "alpha1", "lin_frac2", "eta2", "alpha2", "beta1", "beta2", "adam_eps", "ik_lambda",
                 "ik_noise", "mid_noise", "sat_eps"):
        setattr(p, name, float(getattr(pr, name)))
    return p


class Problem:
    """One problem uploaded to the current device (synth.Problem + synth.Params)."""

    def __init__(self, prob, params):
        L = load()
        self.prob, self.params = prob, params
        self.B = prob.B
        # motion segments: transit and transfer per block, or one point-to-point motion
        self.NS = 1 if int(prob.mode) == MODE_P2P else 2 * prob.B
        self._chain = chain_desc(prob)
        self._params = params_desc(params)
        self._init = np.ascontiguousarray(prob.block_init, dtype=np.float64)
        self._goal = np.ascontiguousarray(np.nan_to_num(prob.goal), dtype=np.float64)
        sk = SkeletonDesc()
        sk.n_blocks, sk.mode = prob.B, int(prob.mode)
        sk.block_edge, sk.block_margin = float(prob.h), float(prob.block_margin)
        sk.block_init = self._init.ctypes.data_as(c_vp)
        sk.goal = self._goal.ctypes.data_as(c_vp)
        sk.grasp[:] = [float(v) for v in np.asarray(prob.grasp, dtype=np.float64).ravel()]
        sk.region[:] = [float(v) for v in prob.table]
        if getattr(prob, "pack_cells", None) is not None:
            self._cells = np.ascontiguousarray(prob.pack_cells, dtype=np.int32)
            self._off = np.ascontiguousarray(prob.pack_off, dtype=np.float64)
            sk.pack_cells = self._cells.ctypes.data_as(c_vp)
            sk.pack_off = self._off.ctypes.data_as(c_vp)
        sk.sample_yaw_steps = int(getattr(prob, "sample_yaw_steps", 0))
        if getattr(prob, "p2p_goal", None) is not None:
            self._p2p_goal = np.ascontiguousarray(prob.p2p_goal, dtype=np.float64)
            sk.p2p_goal = self._p2p_goal.ctypes.data_as(c_vp)
        self._skel = sk
        link = np.ascontiguousarray(prob.sph_link, dtype=np.int32)
        cen = np.ascontiguousarray(prob.sph_c, dtype=np.float64)
        rad = np.ascontiguousarray(prob.sph_r, dtype=np.float64)
        boxes = np.ascontiguousarray(prob.boxes, dtype=np.float64).reshape(-1, 6)
        h = c_vp()
        _check(L.spasm_problem_create(ctypes.byref(self._chain), prob.S, link.ctypes.data_as(c_vp),
                                      cen.ctypes.data_as(c_vp), rad.ctypes.data_as(c_vp), prob.O,
                                      boxes.ctypes.data_as(c_vp) if prob.O else None, ctypes.byref(sk),
                                      ctypes.byref(self._params), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().spasm_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- stage 1 ----------------------------------------------------------------------
    def sample(self, N, seed, rnd=0, out=None):
        x = out if out is not None else _empty(N, self.B, 3)
        _check(load().spasm_sample(self.handle, N, seed, rnd, _dev(x, (N, self.B, 3), name="x"), _stream()))
        return x

    def place_cost(self, x, phase=PHASE_LIN, grad=True):
        N = x.shape[0]
        cost, viol = _empty(N), _empty(N)
        gx = _empty(N, self.B, 3) if grad else None
        _check(load().spasm_cost_grad(self.handle, STAGE_PLACE, phase, N, 0, _dev(x, (N, self.B, 3), name="x"),
                                      None, _dev(cost), _dev(viol), _dev(gx), None, _stream()))
        return cost, viol, gx

    def place_optimize(self, x, k_begin, k_end):
        """In place on x; returns the quadratic-phase cost and violation of the result."""
        N = x.shape[0]
        cost, viol = _empty(N), _empty(N)
        _check(load().spasm_optimize(self.handle, STAGE_PLACE, N, 0, _dev(x, (N, self.B, 3), name="x"), None, None,
                                     k_begin, k_end, 0, _dev(cost), _dev(viol), _stream()))
        return cost, viol

    def place_workspace(self, N, M):
        n = load().spasm_place_workspace(self.handle, N, M)
        if n == 0:
            raise SpasmError(f"unsupported placement round shape N={N} M={M}")
        return torch.empty(n, dtype=torch.uint8, device="cuda")

    def place_round(self, N, M, seed, rnd=0, work=None):
        """One placement-only round: returns (x [M, B, 3] satisfying first, cost [M], viol [M],
        nsat [1] int32), all on the device."""
        work = self.place_workspace(N, M) if work is None else work
        x, cost, viol = _empty(M, self.B, 3), _empty(M), _empty(M)
        nsat = _empty(1, dtype=torch.int32)
        _check(load().spasm_place_round(self.handle, N, M, seed, rnd, _dev(work, dtype=torch.uint8), work.numel(),
                                        _dev(x), _dev(cost), _dev(viol), _dev(nsat, dtype=torch.int32), _stream()))
        return x, cost, viol, nsat

    def sample_placements(self, N, M, seed, rnd=0, work=None):
        """Alg. 1 lines 1-4: the M lowest-cost of N samples (x [M, B, 3], cost [M], viol [M],
        linear phase), on the device."""
        need = load().spasm_sample_placements_workspace(self.handle, N, M)
        if need == 0:
            raise SpasmError(f"unsupported sample shape N={N} M={M}")
        work = torch.empty(need, dtype=torch.uint8, device="cuda") if work is None else work
        x, cost, viol = _empty(M, self.B, 3), _empty(M), _empty(M)
        _check(load().spasm_sample_placements(self.handle, N, M, seed, rnd, _dev(work, dtype=torch.uint8),
                                              work.numel(), _dev(x), _dev(cost), _dev(viol), _stream()))
        return x, cost, viol

    def stage1(self, N, M, seed, work=None):
        """Alg. 1 lines 1-23 (the solve's stage 1): (pose [M, B, 4] satisfying first, cost [M],
        viol [M] quadratic phase, info [2] int32 = satisfying count, rounds), on the device."""
        need = load().spasm_stage1_workspace(self.handle, N, M)
        if need == 0:
            _check(-1)
        work = torch.empty(need, dtype=torch.uint8, device="cuda") if work is None else work
        pose, cost, viol = _empty(M, self.B, 4), _empty(M), _empty(M)
        info = _empty(2, dtype=torch.int32)
        _check(load().spasm_stage1(self.handle, N, M, seed, _dev(work, dtype=torch.uint8), work.numel(), _dev(pose),
                                   _dev(cost), _dev(viol), _dev(info, dtype=torch.int32), _stream()))
        return pose, cost, viol, info

    # ---- stage 2 ----------------------------------------------------------------------
    def traj_cost(self, q, pose, phase=PHASE_LIN, grad=True):
        P, NS, W, _ = q.shape
        cost, viol = _empty(P), _empty(P)
        gq = _empty(P, NS, W, 7) if grad else None
        gp = _empty(P, self.B, 4) if grad else None
        _check(load().spasm_cost_grad(self.handle, STAGE_TRAJ, phase, P, W,
                                      _dev(q, (P, self.NS, W, 7), name="q"), _dev(pose, (P, self.B, 4), name="pose"),
                                      _dev(cost), _dev(viol), _dev(gq), _dev(gp), _stream()))
        return cost, viol, gq, gp

    def traj_cost_al(self, q, pose, lam, phase=PHASE_LIN, grad=True):
        """Stage-2 cost with the multiplier terms lambda . e; lam [P, B, 15]."""
        P, NS, W, _ = q.shape
        cost, viol = _empty(P), _empty(P)
        gq = _empty(P, NS, W, 7) if grad else None
        gp = _empty(P, self.B, 4) if grad else None
        _check(load().spasm_cost_grad_al(self.handle, phase, P, W, _dev(q, (P, self.NS, W, 7), name="q"),
                                         _dev(pose, (P, self.B, 4), name="pose"), _dev(lam, (P, self.B, 15), name="lam"),
                                         _dev(cost), _dev(viol), _dev(gq), _dev(gp), _stream()))
        return cost, viol, gq, gp

    def traj_adjoint(self, q, pose, gout, phase=PHASE_LIN):
        P, NS, W, _ = q.shape
        gq, gp = _empty(P, NS, W, 7), _empty(P, self.B, 4)
        _check(load().spasm_cost_adjoint(self.handle, phase, P, W, _dev(q, (P, self.NS, W, 7), name="q"),
                                         _dev(pose, (P, self.B, 4), name="pose"), _dev(gout, (P,), name="gout"),
                                         _dev(gq), _dev(gp), _stream()))
        return gq, gp

    def opt_state(self, P, W):
        """Optimiser state rows: Adam m and v, then the 15B multipliers with al_every > 0."""
        al = 15 * self.B if int(getattr(self.params, "al_every", 0)) > 0 else 0
        return torch.zeros(P, 2 * (2 * self.B * W * 7 + 4 * self.B) + al, dtype=torch.float32, device="cuda")

    def traj_optimize(self, q, pose, opt, k_begin, k_end, K_total, want_cost=True):
        """In place on q, pose and opt (Adam moments)."""
        P, NS, W, _ = q.shape
        cost = _empty(P) if want_cost else None
        viol = _empty(P) if want_cost else None
        _check(load().spasm_optimize(self.handle, STAGE_TRAJ, P, W, _dev(q, (P, self.NS, W, 7), name="q"),
                                     _dev(pose, (P, self.B, 4), name="pose"), _dev(opt, name="opt"), k_begin, k_end,
                                     K_total, _dev(cost), _dev(viol), _stream()))
        return cost, viol

    # ---- lift / seed ---------------------------------------------------------------------
    def ik_iterate(self, kind, target, q, iters):
        n = q.shape[0]
        _check(load().spasm_ik_iterate(self.handle, kind, n, _dev(target, (n, 4), name="target"),
                                       _dev(q, (n, 7), name="q"), iters, _stream()))
        return q

    def ik_lift(self, pose, seed, iters=None):
        P = pose.shape[0]
        qg, qp = _empty(P, self.B, 7), _empty(P, self.B, 7)
        _check(load().spasm_ik_lift(self.handle, P, _dev(pose, (P, self.B, 4), name="pose"), seed,
                                    self.params.ik_iters if iters is None else iters, _dev(qg), _dev(qp), _stream()))
        return qg, qp

    def traj_init(self, qg, qp, W, seed, pose, P=None):
        """Seeds [P, NS, W, 7]; a point-to-point problem takes qg = qp = pose = None and P."""
        P = qg.shape[0] if qg is not None else P
        q = _empty(P, self.NS, W, 7)
        _check(load().spasm_traj_init(self.handle, P, W, _dev(qg, (P, self.B, 7), name="qg"),
                                      _dev(qp, (P, self.B, 7), name="qp"), _dev(pose, (P, self.B, 4), name="pose"),
                                      seed, _dev(q), _stream()))
        return q

    # ---- whole method ----------------------------------------------------------------------
    def config_desc(self, cfg) -> SolveConfigDesc:
        c = SolveConfigDesc()
        c.N1, c.M, c.W, c.K, c.seed = int(cfg.N1), int(cfg.M), int(cfg.W), int(cfg.K), int(cfg.seed)
        return c

    def workspace_bytes(self, cfg) -> int:
        c = self.config_desc(cfg)
        n = load().spasm_solve_workspace(self.handle, ctypes.byref(c))
        if n == 0:
            raise SpasmError(load().spasm_last_error().decode())
        return int(n)

    def footprint(self, cfg) -> int:
        """Device bytes of one plain solve: workspace plus outputs."""
        c = self.config_desc(cfg)
        n = load().spasm_solve_footprint(self.handle, ctypes.byref(c))
        if n == 0:
            raise SpasmError(load().spasm_last_error().decode())
        return int(n)

    def make_workspace(self, cfg):
        n = self.workspace_bytes(cfg)
        return torch.empty((n + 255) // 4, dtype=torch.float32, device="cuda")

    def solve(self, cfg, work=None, best_q=None, best_pose=None):
        c = self.config_desc(cfg)
        if work is None:
            work = self.make_workspace(cfg)
        if best_q is None:
            best_q = _empty(self.NS, cfg.W, 7)
        if best_pose is None:
            best_pose = _empty(self.B, 4)
        res = ResultDesc()
        _check(load().spasm_solve(self.handle, ctypes.byref(c), _dev(work, name="work"), work.numel() * 4,
                                  _dev(best_q, (self.NS, cfg.W, 7), name="best_q"),
                                  _dev(best_pose, (self.B, 4), name="best_pose"), ctypes.byref(res), _stream()))
        out = {f: getattr(res, f) for f, _ in ResultDesc._fields_}
        return out, best_q, best_pose

    def solve_ttfs(self, cfg, check_every, max_attempts, work=None, best_q=None, best_pose=None):
        """Time to first solution: returns (result dict with 'attempts' and 'iters', best_q, best_pose)."""
        c = self.config_desc(cfg)
        if work is None:
            n = load().spasm_solve_ttfs_workspace(self.handle, ctypes.byref(c))
            if n == 0:
                _check(-1)
            work = torch.empty(n, dtype=torch.uint8, device="cuda")
        if best_q is None:
            best_q = _empty(self.NS, cfg.W, 7)
        if best_pose is None:
            best_pose = _empty(self.B, 4)
        res, att, its = ResultDesc(), c_i32(), c_i32()
        _check(load().spasm_solve_ttfs(self.handle, ctypes.byref(c), check_every, max_attempts,
                                       _dev(work, dtype=torch.uint8, name="work"), work.numel(),
                                       _dev(best_q, (self.NS, cfg.W, 7), name="best_q"),
                                       _dev(best_pose, (self.B, 4), name="best_pose"), ctypes.byref(res),
                                       ctypes.byref(att), ctypes.byref(its), _stream()))
        out = {f: getattr(res, f) for f, _ in ResultDesc._fields_}
        out["attempts"], out["iters"] = att.value, its.value
        return out, best_q, best_pose


class Server:
    """Continuous-batching server (spasm_server_*): submit requests, call step() to admit,
    advance and retire, poll() completions.  Keeps each request's problem and output
    tensors alive until its completion has been polled."""

    def __init__(self, hbm_budget, max_slots=64, iters_per_step=25):
        h = c_vp()
        _check(load().spasm_server_create(int(hbm_budget), int(max_slots), int(iters_per_step), ctypes.byref(h)))
        self.handle = h
        self._live = {}

    @staticmethod
    def footprint(problem, cfg):
        c = problem.config_desc(cfg)
        return int(load().spasm_server_footprint(problem.handle, ctypes.byref(c)))

    def submit(self, problem, cfg, req_id):
        c = problem.config_desc(cfg)
        best_q = _empty(2 * problem.B, cfg.W, 7)
        best_pose = _empty(problem.B, 4)
        _check(load().spasm_server_submit(self.handle, problem.handle, ctypes.byref(c), int(req_id),
                                          _dev(best_q), _dev(best_pose)))
        self._live[int(req_id)] = (problem, best_q, best_pose)

    def step(self):
        na, npend = c_i32(), c_i32()
        _check(load().spasm_server_step(self.handle, ctypes.byref(na), ctypes.byref(npend)))
        return na.value, npend.value

    def poll(self, max_n=256):
        arr = (CompletionDesc * max_n)()
        n = c_i32()
        _check(load().spasm_server_poll(self.handle, arr, max_n, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            c = arr[i]
            res = {f: getattr(c.result, f) for f, _ in ResultDesc._fields_}
            _, bq, bp = self._live.pop(int(c.req_id))
            out.append({"req_id": int(c.req_id), "status": c.status, "steps": c.steps, "result": res,
                        "best_q": bq, "best_pose": bp})
        return out

    def close(self):
        if getattr(self, "handle", None):
            load().spasm_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def select_topm(key, M):
    N = key.shape[0]
    idx = _empty(M, dtype=torch.int32)
    _check(load().spasm_select_topm(N, _dev(key, (N,), name="key"), M, _dev(idx, dtype=torch.int32), _stream()))
    return idx


def select_topm_large(key, M, work=None):
    """select_topm for up to 2^20 keys (radix select); allocates its workspace if not given."""
    N = key.shape[0]
    need = load().spasm_select_topm_workspace(N, M)
    if work is None and need:
        work = torch.empty(need, dtype=torch.uint8, device="cuda")
    idx = _empty(M, dtype=torch.int32)
    _check(load().spasm_select_topm_large(N, _dev(key, (N,), name="key"), M, _dev(idx, dtype=torch.int32),
                                          _dev(work, dtype=torch.uint8) if need else None,
                                          work.numel() if need else 0, _stream()))
    return idx


def order(cost, viol, eps):
    n = cost.shape[0]
    out = _empty(n, dtype=torch.int32)
    nsat = _empty(1, dtype=torch.int32)
    _check(load().spasm_order(n, _dev(cost, (n,), name="cost"), _dev(viol, (n,), name="viol"), float(eps),
                              _dev(out, dtype=torch.int32), _dev(nsat, dtype=torch.int32), _stream()))
    return out, nsat


class SpasmCost(torch.autograd.Function):
    """Stage-2 cost (Appendix B C_trajopt) as a differentiable function of the joint
    trajectories q [P, 2B, W, 7] and block poses [P, B, 4]; forward runs the cost-only
    kernel, backward the hand-written adjoint kernel."""

    @staticmethod
    def forward(ctx, q, pose, problem, phase=PHASE_LIN):
        q, pose = q.contiguous(), pose.contiguous()
        cost, _, _, _ = problem.traj_cost(q, pose, phase, grad=False)
        ctx.save_for_backward(q, pose)
        ctx.problem, ctx.phase = problem, phase
        return cost

    @staticmethod
    def backward(ctx, gout):
        q, pose = ctx.saved_tensors
        gq, gp = ctx.problem.traj_adjoint(q, pose, gout.contiguous().to(torch.float32), ctx.phase)
        return gq, gp, None, None
