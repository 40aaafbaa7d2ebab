"""Continuous-batching server (through the C ABI): requests that arrive while others run
are admitted as slots and arena space free up, run together with them, and each result
equals the solo ot_solve result bit for bit (same parameters and tile shapes)."""
import time

import numpy as np
import pytest

import paper_2407_19689_amd as P
from tests.test_gpu_parity import assert_matches_oracle
from workloads import generators as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P._abi.load()
    torch.cuda.set_device(0)


def mixed_requests(count, seed=7):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        r = rng.uniform()
        tol = float(rng.choice([1e-4, 1e-6]))
        if r < 0.2:
            inst = gen.grid_pair(9000 + i, int(rng.integers(6, 24)), tol=tol)
        elif r < 0.6:
            inst = gen.points_sqeuclid(9000 + i, int(rng.integers(20, 700)), int(rng.integers(20, 700)),
                                       tol=tol)
        else:
            inst = gen.points_sqeuclid(9000 + i, int(rng.integers(600, 1600)),
                                       int(rng.integers(600, 1600)), tol=tol)
        out.append(inst)
    return out


def test_server_results_equal_solo_and_overlap():
    prm = P.params(tol=1e-4, precision=P.OT_PREC_FP32, time_limit_s=60.0)
    insts = mixed_requests(14)
    outs = []
    with P.Server(2 << 30, max_active=6, prm=prm) as srv:
        tickets = []
        for k, inst in enumerate(insts):
            pr, out = P.problem_from_instance(inst, precision=P.OT_PREC_FP32, tol=inst.tol)
            st, t = srv.submit(pr)
            assert st == P.OT_OK, P.ot_last_error()
            tickets.append(t)
            outs.append(out)
            if k % 3 == 2:
                time.sleep(0.01)          # later requests arrive while earlier ones run
        assert srv.drain(120.0) == P.OT_OK
        done = {d["ticket"]: d for d in srv.poll(64)}
        stats = srv.stats()
    assert stats["completed"] == len(insts) and stats["max_running"] > 1
    assert stats["max_running"] <= 6
    # continuous batching: some request was admitted before an earlier one finished
    ordered = [done[t] for t in tickets]
    assert any(ordered[j]["t_admit"] < ordered[i]["t_done"]
               for i in range(len(ordered)) for j in range(i + 1, len(ordered)))
    for inst, t, out in zip(insts, tickets, outs):
        d = done[t]
        assert d["status"] == P.OT_OK
        st, res, solo = P.solve_instance(inst, prm, tol=inst.tol)
        assert st == P.OT_OK
        assert d["iterations"] == res["iterations"] and d["restarts"] == res["restarts"]
        assert d["objective"] == res["objective"]
        assert np.array_equal(out["X"].cpu().numpy(), solo["X"].cpu().numpy())
        assert np.array_equal(out["u"].cpu().numpy(), solo["u"].cpu().numpy())
        assert_matches_oracle(inst, d, out, P.OT_PREC_FP32)


def test_server_admission_respects_the_memory_budget():
    prm = P.params(tol=1e-4, precision=P.OT_PREC_FP32, time_limit_s=60.0)
    insts = [gen.points_sqeuclid(500 + i, 1500, 1500, tol=1e-4) for i in range(6)]
    one = P.ot_workspace_size(P.problem_from_instance(insts[0])[0], prm)
    budget = int(2.5 * one)       # room for two instances at a time
    with P.Server(budget, max_active=8, prm=prm) as srv:
        for inst in insts:
            pr, _ = P.problem_from_instance(inst, want_plan=False)
            assert srv.submit(pr)[0] == P.OT_OK
        assert srv.drain(120.0) == P.OT_OK
        stats = srv.stats()
        done = srv.poll(64)
    assert all(d["status"] == P.OT_OK for d in done)
    assert stats["arena_peak"] <= budget
    assert 1 <= stats["max_running"] <= 2


def test_server_rejects_a_request_larger_than_its_budget():
    prm = P.params(tol=1e-4)
    with P.Server(8 << 20, max_active=4, prm=prm) as srv:
        inst = gen.points_sqeuclid(1, 2000, 2000)
        pr, _ = P.problem_from_instance(inst, want_plan=False)
        st, _ = srv.submit(pr)
        assert st == P.OT_ERR_BUSY
        small = gen.points_sqeuclid(2, 40, 50, tol=1e-4)
        pr2, out2 = P.problem_from_instance(small)
        assert srv.submit(pr2)[0] == P.OT_OK
        assert srv.drain(60.0) == P.OT_OK
        (d,) = srv.poll(4)
        assert d["status"] == P.OT_OK and d["rel_kkt"] <= 1e-4
