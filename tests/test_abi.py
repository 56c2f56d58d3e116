"""CPU checks of the C-ABI library: it loads, exports every entry point the header
declares, and rejects bad arguments before touching the device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from conftest import ROOT


def _declared():
    text = open(os.path.join(ROOT, "include", "spasm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spasm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("spasm_problem_create", "spasm_problem_destroy", "spasm_sample", "spasm_cost_grad",
              "spasm_cost_adjoint", "spasm_optimize", "spasm_select_topm", "spasm_order", "spasm_ik_iterate",
              "spasm_ik_lift", "spasm_traj_init", "spasm_solve", "spasm_solve_workspace", "spasm_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2510_07674_amd import spasm
    L = spasm.load()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) == set(spasm.SYMBOLS)


def _problem_args(prob, params):
    from paper_2510_07674_amd import spasm
    chain = spasm.chain_desc(prob)
    pr = spasm.params_desc(params)
    init = np.ascontiguousarray(prob.block_init, dtype=np.float64)
    goal = np.ascontiguousarray(np.nan_to_num(prob.goal), dtype=np.float64)
    sk = spasm.SkeletonDesc()
    sk.n_blocks, sk.mode = prob.B, prob.mode
    sk.block_edge, sk.block_margin = prob.h, prob.block_margin
    sk.block_init = init.ctypes.data_as(ctypes.c_void_p)
    sk.goal = goal.ctypes.data_as(ctypes.c_void_p)
    sk.grasp[:] = list(np.asarray(prob.grasp, float).ravel())
    sk.region[:] = list(prob.table)
    link = np.ascontiguousarray(prob.sph_link, np.int32)
    cen = np.ascontiguousarray(prob.sph_c, np.float64)
    rad = np.ascontiguousarray(prob.sph_r, np.float64)
    boxes = np.ascontiguousarray(prob.boxes, np.float64)
    return dict(chain=chain, pr=pr, sk=sk, link=link, cen=cen, rad=rad, boxes=boxes, keep=(init, goal))


def _create(a, n_sph=None, n_obs=None):
    from paper_2510_07674_amd import spasm
    L = spasm.load()
    h = ctypes.c_void_p()
    vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    rc = L.spasm_problem_create(ctypes.byref(a["chain"]), len(a["rad"]) if n_sph is None else n_sph,
                                vp(a["link"]), vp(a["cen"]), vp(a["rad"]),
                                len(a["boxes"]) if n_obs is None else n_obs, vp(a["boxes"]), ctypes.byref(a["sk"]),
                                ctypes.byref(a["pr"]), ctypes.byref(h))
    return rc, L.spasm_last_error().decode()


@pytest.mark.parametrize("mutate,code", [
    ("nan_dh", -1), ("bad_link", -1), ("link_order", -1), ("neg_radius", -1), ("neg_half", -1),
    ("too_many_blocks", -4), ("bad_mode", -1), ("bad_grasp", -1), ("neg_weight", -1), ("bad_beta", -1),
    ("small_region", -1), ("neg_count", -1), ("no_ik_starts", -1), ("too_many_ik_starts", -1), ("no_mid", -1), ("too_many_mid", -1),
])
def test_problem_create_rejects(mutate, code):
    from paper_2510_07674_amd import synth
    prob, params, _ = synth.config("tower4", 0)
    a = _problem_args(prob, params)
    n_sph = None
    if mutate == "nan_dh":
        a["chain"].dh[4] = math.nan
    elif mutate == "bad_link":
        a["link"][3] = 9
    elif mutate == "link_order":
        a["link"][0] = 7
    elif mutate == "neg_radius":
        a["rad"][2] = -0.01
    elif mutate == "neg_half":
        a["boxes"][1, 4] = -0.1
    elif mutate == "too_many_blocks":
        a["sk"].n_blocks = 17
    elif mutate == "bad_mode":
        a["sk"].mode = 5
    elif mutate == "bad_grasp":
        a["sk"].grasp[0] = 2.0
    elif mutate == "neg_weight":
        a["pr"].w[5] = -1.0
    elif mutate == "bad_beta":
        a["pr"].beta2 = 1.0
    elif mutate == "small_region":
        a["sk"].region[1] = a["sk"].region[0] + 0.01
    elif mutate == "neg_count":
        n_sph = -1
    elif mutate == "no_ik_starts":
        a["pr"].ik_restarts = 0
    elif mutate == "too_many_ik_starts":
        a["pr"].ik_restarts = 9
    elif mutate == "no_mid":
        a["pr"].mid_candidates = 0
    elif mutate == "too_many_mid":
        a["pr"].mid_candidates = 9
    rc, msg = _create(a, n_sph=n_sph)
    assert rc == code and msg


def test_selection_size_checks():
    from paper_2510_07674_amd import spasm
    L = spasm.load()
    assert L.spasm_select_topm(0, None, 1, None, None) == -4
    assert L.spasm_select_topm(20000, None, 1, None, None) == -4
    assert L.spasm_select_topm(100, None, 101, None, None) == -1
    assert L.spasm_order(0, None, None, 1e-3, None, None, None) == -4
    assert "outside" in L.spasm_last_error().decode()


def test_null_problem_is_rejected():
    from paper_2510_07674_amd import spasm
    L = spasm.load()
    assert L.spasm_sample(None, 10, 0, 0, None, None) == -1
    assert L.spasm_cost_grad(None, 2, 0, 1, 16, None, None, None, None, None, None, None) == -1
    assert L.spasm_optimize(None, 2, 1, 16, None, None, None, 1, 2, 1, None, None, None) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2510_07674_amd import spasm
    monkeypatch.setattr(spasm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(spasm, "_lib", None)
    with pytest.raises(spasm.SpasmError):
        spasm.load()


def test_topm_and_place_shapes():
    """Radix-select workspace sizes and placement-round shape checks run on the host."""
    from paper_2510_07674_amd import spasm
    L = spasm.load()
    assert L.spasm_select_topm_workspace(16384, 2048) == 0
    # radix select: state (256 B), 2048-bin histogram, two counts per workgroup of 4096
    # keys rounded up to 256 B, M (cost bits, index) survivors
    assert L.spasm_select_topm_workspace(131072, 256) == 256 + 2048 * 4 + 256 + 256 * 8
    assert L.spasm_select_topm_workspace(1 << 20, 8192) == 256 + 2048 * 4 + 2048 + 8192 * 8
    assert L.spasm_select_topm_workspace(1 << 21, 256) == 0          # too many keys
    assert L.spasm_select_topm_workspace(20000, 8193) == 0           # M too large for chunking
    dummy = ctypes.c_void_p(256)
    assert L.spasm_select_topm_large(1 << 21, dummy, 8, dummy, None, 0, None) == -4
    assert L.spasm_select_topm_large(20000, dummy, 8193, dummy, None, 0, None) == -4
    assert L.spasm_select_topm_large(20000, dummy, 0, dummy, None, 0, None) == -1
    assert L.spasm_select_topm_large(20000, dummy, 8, dummy, None, 0, None) == -1   # no workspace
    need = L.spasm_select_topm_workspace(20000, 8)
    assert L.spasm_select_topm_large(20000, dummy, 8, dummy, ctypes.c_void_p(256 + 4), need, None) == -1
    assert "256-byte aligned" in L.spasm_last_error().decode()
    assert L.spasm_place_round(None, 100, 10, 0, 0, None, 0, dummy, None, None, dummy, None) == -1


def test_stage1_and_footprint_need_a_problem():
    """The sampled-placement, whole-stage-1 and footprint calls refuse a NULL problem on the
    host (0 bytes from the sizing calls, SPASM_EINVAL from the others)."""
    from paper_2510_07674_amd import spasm
    L = spasm.load()
    dummy = ctypes.c_void_p(256)
    assert L.spasm_sample_placements_workspace(None, 100, 10) == 0
    assert L.spasm_sample_placements(None, 100, 10, 0, 0, dummy, 1 << 20, dummy, None, None, None) == -1
    assert L.spasm_stage1_workspace(None, 100, 10) == 0
    rc = L.spasm_stage1(None, 100, 10, 0, dummy, 1 << 20, dummy, None, None, dummy, None)
    assert rc == -1 and "NULL" in L.spasm_last_error().decode()
    cfg = spasm.SolveConfigDesc(4096, 1024, 32, 200, 0)
    assert L.spasm_solve_footprint(None, ctypes.byref(cfg)) == 0


@pytest.mark.parametrize("mutate", [
    "pack_no_cells", "pack_zero_cells", "pack_nine_cells", "pack_nan_offset", "yaw_steps_high", "yaw_steps_neg",
    "p2p_two_blocks", "p2p_no_goal", "p2p_goal_outside", "p2p_start_outside", "al_every_neg", "al_rho_neg",
    "al_rho_nan",
])
def test_problem_create_rejects_mode_options(mutate):
    """Host validation of the packing, point-to-point and augmented-Lagrangian options:
    every bad description is refused with SPASM_EINVAL before any device call."""
    from paper_2510_07674_amd import synth
    if mutate.startswith("pack") or mutate.startswith("yaw"):
        prob, params, _ = synth.config("tetris5", 0)
    elif mutate.startswith("p2p"):
        prob, params, _ = synth.config("p2p", synth.p2p_seeds()[0])
    else:
        prob, params, _ = synth.config("tower4", 0)
    a = _problem_args(prob, params)
    cells = np.ascontiguousarray(prob.pack_cells if prob.pack_cells is not None else np.ones(prob.B), np.int32)
    off = np.ascontiguousarray(prob.pack_off if prob.pack_off is not None else np.zeros((prob.B, 8, 2)), np.float64)
    goal = np.ascontiguousarray(prob.p2p_goal if prob.p2p_goal is not None else np.zeros(7), np.float64)
    a["keep"] = a["keep"] + (cells, off, goal)
    if prob.mode == synth.MODE_PACK:
        a["sk"].pack_cells = cells.ctypes.data_as(ctypes.c_void_p)
        a["sk"].pack_off = off.ctypes.data_as(ctypes.c_void_p)
        a["sk"].sample_yaw_steps = 4
    if prob.mode == synth.MODE_P2P:
        a["sk"].p2p_goal = goal.ctypes.data_as(ctypes.c_void_p)
    if mutate == "pack_no_cells":
        a["sk"].pack_cells = None
    elif mutate == "pack_zero_cells":
        cells[1] = 0
    elif mutate == "pack_nine_cells":
        cells[2] = 9
    elif mutate == "pack_nan_offset":
        off[0, 1, 0] = math.nan
    elif mutate == "yaw_steps_high":
        a["sk"].sample_yaw_steps = 65
    elif mutate == "yaw_steps_neg":
        a["sk"].sample_yaw_steps = -1
    elif mutate == "p2p_two_blocks":
        a["sk"].n_blocks = 2
        init2 = np.zeros((2, 4))
        a["keep"] = a["keep"] + (init2,)
        a["sk"].block_init = init2.ctypes.data_as(ctypes.c_void_p)
    elif mutate == "p2p_no_goal":
        a["sk"].p2p_goal = None
    elif mutate == "p2p_goal_outside":
        goal[3] = 3.0
    elif mutate == "p2p_start_outside":
        a["chain"].q_home[5] = -3.0
    elif mutate == "al_every_neg":
        a["pr"].al_every = -1
    elif mutate == "al_rho_neg":
        a["pr"].al_rho = -0.5
    elif mutate == "al_rho_nan":
        a["pr"].al_rho = math.nan
    rc, msg = _create(a)
    assert rc == -1 and msg, (rc, msg)


def test_static_topm_size_checks():
    """The allocation-free selection refuses shapes beyond its static scratch on the host;
    the scratch holds the largest workspace the radix select can ask for."""
    from paper_2510_07674_amd import spasm
    L = spasm.load()
    dummy = ctypes.c_void_p(256)
    assert L.spasm_select_topm_static((1 << 20) + 1, dummy, 8, dummy, None) == -4
    assert L.spasm_select_topm_static(20000, dummy, 8193, dummy, None) == -4
    assert L.spasm_select_topm_static(100, dummy, 101, dummy, None) == -1
    assert L.spasm_select_topm_static(100, None, 10, dummy, None) == -1
    assert L.spasm_select_topm_static_bytes() == L.spasm_select_topm_workspace(1 << 20, 8192)
