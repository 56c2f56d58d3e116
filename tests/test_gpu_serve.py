"""Serving (continuous batching) on the GPU: a request's result does not depend on what
else is batched with it, it equals the plain one-solve-per-launch result, and admission
follows the HBM budget."""
import numpy as np
import pytest
import torch

from paper_2510_07674_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    from paper_2510_07674_amd import spasm
    spasm.load()
    return spasm


def _req(sp, seed, B, O, W, M, K, mode=synth.MODE_TOWER):
    prob = synth.make_problem(seed, B=B, O=O, S=42, mode=mode)
    pr = synth.Params()
    N1 = 0 if mode == synth.MODE_FIXED else 4 * M
    cfg = synth.SolveConfig(N1=N1, M=M, W=W, K=K, seed=seed)
    return sp.Problem(prob, pr), cfg


def _drain(srv, limit=500):
    out = {}
    for _ in range(limit):
        active, pending = srv.step()
        for c in srv.poll():
            out[c["req_id"]] = c
        if active == 0 and pending == 0:
            break
    return out


def _mix(sp):
    return [_req(sp, 1, 2, 20, 16, 128, 60), _req(sp, 2, 3, 30, 32, 96, 45), _req(sp, 3, 1, 10, 16, 64, 50, synth.MODE_FIXED),
            _req(sp, 4, 5, 15, 16, 160, 80), _req(sp, 5, 2, 0, 32, 64, 26)]


def test_result_same_alone_and_in_mix(sp):
    reqs = _mix(sp)
    budget = 2 << 30
    alone = {}
    for i, (dev, cfg) in enumerate(reqs):
        srv = sp.Server(budget, max_slots=8, iters_per_step=10)
        srv.submit(dev, cfg, i)
        alone.update(_drain(srv))
        srv.close()
    srv = sp.Server(budget, max_slots=8, iters_per_step=10)
    srv.submit(*reqs[1], 1)
    srv.submit(*reqs[2], 2)
    srv.step()                      # 1 and 2 are running when the others arrive
    srv.submit(*reqs[0], 0)
    srv.step()
    srv.submit(*reqs[3], 3)
    srv.submit(*reqs[4], 4)
    mixed = {}
    for c in srv.poll():
        mixed[c["req_id"]] = c
    mixed.update(_drain(srv))
    srv.close()
    assert sorted(mixed) == list(range(len(reqs)))
    for i in range(len(reqs)):
        a, m = alone[i], mixed[i]
        assert a["status"] == 0 and m["status"] == 0
        assert torch.equal(a["best_q"], m["best_q"]) and torch.equal(a["best_pose"], m["best_pose"]), i
        assert a["result"]["viol"] == m["result"]["viol"] and a["result"]["best"] == m["result"]["best"]
    # same as the plain path (fused single launch per solve)
    for i, (dev, cfg) in enumerate(reqs):
        res, bq, bp = dev.solve(cfg)
        assert torch.equal(bq, mixed[i]["best_q"]) and torch.equal(bp, mixed[i]["best_pose"]), i
        assert res["viol"] == mixed[i]["result"]["viol"] and res["n_sat"] == mixed[i]["result"]["n_sat"]


@pytest.mark.parametrize("B,M", [(5, 1024), (10, 512)])
def test_reordered_plain_solve_equals_served(sp, B, M):
    """1024 particles of 5 waves (or 512 of 10 waves, whose launches take the 768-thread
    register bound) do not all fit on the chip at once, so the plain solve launches them
    costliest first, while the serving launch takes them in natural order; every particle
    computes the same on any workgroup, so the results are identical."""
    dev, cfg = _req(sp, 7, B, 30, 32, M, 30)
    srv = sp.Server(2 << 30, max_slots=4, iters_per_step=10)
    srv.submit(dev, cfg, 0)
    out = _drain(srv)
    srv.close()
    res, bq, bp = dev.solve(cfg)
    assert out[0]["status"] == 0
    assert torch.equal(bq, out[0]["best_q"]) and torch.equal(bp, out[0]["best_pose"])
    assert res["viol"] == out[0]["result"]["viol"] and res["n_sat"] == out[0]["result"]["n_sat"]


def test_admission_follows_budget(sp):
    reqs = [_req(sp, 11, 2, 10, 16, 128, 40), _req(sp, 12, 2, 10, 16, 128, 40)]
    need = sp.Server.footprint(*reqs[0])
    assert need > 0 and need == sp.Server.footprint(*reqs[1])
    srv = sp.Server(need + 4096, max_slots=8, iters_per_step=10)   # room for one at a time
    srv.submit(*reqs[0], 0)
    srv.submit(*reqs[1], 1)
    active, pending = srv.step()
    assert active == 1 and pending == 1
    done = _drain(srv)
    assert sorted(done) == [0, 1]
    # a request alone: its admission step runs the prefix and a first chunk -- 10
    # iterations while its class is untimed, else as many as fit 2 ms -- and each later step
    # at least 10 more: 2 to 4 steps for the first request's 40, 1 to 4 for the second's
    assert 2 <= done[0]["steps"] <= 4 and 1 <= done[1]["steps"] <= 4
    big = _req(sp, 13, 4, 10, 32, 512, 40)
    with pytest.raises(sp.SpasmError):
        srv.submit(*big, 2)
    srv.close()


def test_slot_limit_and_many_classes(sp):
    reqs = [_req(sp, 20 + i, 1 + i % 4, 5 * i, 16 if i % 2 else 32, 64, 20 + 5 * i) for i in range(9)]
    srv = sp.Server(4 << 30, max_slots=3, iters_per_step=7)
    for i, r in enumerate(reqs):
        srv.submit(*r, i)
    active, pending = srv.step()
    assert active == 3 and pending == 6            # no request finishes in one step (K >= 20 > 7)
    done = _drain(srv)
    assert sorted(done) == list(range(9))
    assert all(c["status"] == 0 for c in done.values())
    srv.close()
