"""ot_solve_noalloc (the entry point for callers that cannot allocate) against ot_solve,
through the C ABI: two calls in a row on the library's static device array, the second
with a smaller problem, each equal to ot_solve's result for the same problem bit for bit
(same kernels, same tile shapes, same arithmetic); a problem beyond the array's size is
refused with OT_ERR_OOM before any device work."""
import numpy as np
import pytest

import paper_2407_19689_amd as P
from workloads import generators as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P._abi.load()
    torch.cuda.set_device(0)


def run(fn, inst, prm, dense=False, store=0, trace_cap=0):
    pr, out = P.problem_from_instance(inst, precision=prm.precision, store=store, dense=dense,
                                      tol=inst.tol, trace_cap=trace_cap)
    st, res = fn(pr, prm)
    torch.cuda.synchronize()
    r = res.as_dict()
    arrays = {k: v.cpu().numpy() for k, v in out.items()}
    if trace_cap:
        arrays["trace"] = pr.trace(res.trace_len)
    return st, r, arrays


def assert_same(a, b):
    sa, ra, oa = a
    sb, rb, ob = b
    assert sa == sb
    for k in ("iterations", "passes", "restarts", "kernel_passes", "objective", "rel_kkt",
              "returned_average", "verify_retries"):
        assert ra[k] == rb[k], (k, ra[k], rb[k])
    for k in ("X", "u", "v"):
        assert np.array_equal(oa[k], ob[k]), k
    if "trace" in oa:
        assert oa["trace"] == ob["trace"]


@pytest.mark.parametrize("prec", [P.OT_PREC_FP32, P.OT_PREC_FP64])
def test_two_calls_in_a_row_equal_ot_solve(prec):
    prm = P.params(tol=1e-6, precision=prec, time_limit_s=60.0)
    big = gen.grid_pair(300, 32, tol=1e-6)                 # 1024 x 1024, whole-GPU path
    small = gen.points_sqeuclid(301, 150, 230, tol=1e-6)   # smaller, whole-GPU path
    for inst in (big, small):
        a = run(P.ot_solve_noalloc, inst, prm, trace_cap=64)
        assert a[0] == P.OT_OK, P.ot_last_error()
        b = run(P.ot_solve, inst, prm, trace_cap=64)
        assert_same(a, b)


def test_resident_dense_host_cost_and_stored_cost():
    """A small instance (one work-group runs it), a dense cost in host memory (staged through
    the array), and a stored regenerated cost, each equal to ot_solve's result."""
    prm = P.params(tol=1e-6, precision=P.OT_PREC_FP32, time_limit_s=60.0)
    tiny = gen.points_sqeuclid(302, 40, 50, tol=1e-6)
    assert_same(run(P.ot_solve_noalloc, tiny, prm), run(P.ot_solve, tiny, prm))
    inst = gen.gmm_euclid(303, 200, 330, tol=1e-5)
    for store in (0, 1):
        assert_same(run(P.ot_solve_noalloc, inst, prm, store=store), run(P.ot_solve, inst, prm, store=store))
    C = inst.dense_cost()
    f, g = inst.f, inst.g
    outs = []
    for fn in (P.ot_solve_noalloc, P.ot_solve):
        X = torch.zeros((inst.m, inst.n), dtype=torch.float32, device="cuda")
        u = torch.zeros(inst.m, dtype=torch.float64, device="cuda")
        v = torch.zeros(inst.n, dtype=torch.float64, device="cuda")
        pr = P.problem(P.OT_COST_DENSE, inst.m, inst.n, f, g, C=C, X_out=X, u_out=u, v_out=v)
        st, res = fn(pr, prm)
        torch.cuda.synchronize()
        assert st == P.OT_OK, P.ot_last_error()
        outs.append((res.iterations, res.objective, X.cpu().numpy(), u.cpu().numpy()))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][2], outs[1][2]) and np.array_equal(outs[0][3], outs[1][3])


def test_limits_and_errors_match_ot_solve():
    prm = P.params(tol=1e-9, precision=P.OT_PREC_FP32, max_iters=7, time_limit_s=60.0)
    inst = gen.points_sqeuclid(304, 90, 70, tol=1e-9)
    a = run(P.ot_solve_noalloc, inst, prm)
    assert a[0] == P.OT_NOT_CONVERGED
    assert_same(a, run(P.ot_solve, inst, prm))
    # beyond the array: refused with the size in the message
    huge = gen.grid_pair(305, 96)       # 9216 x 9216 FP32: five plans of 340 MB
    pr, _ = P.problem_from_instance(huge, want_plan=False)
    st, _ = P.ot_solve_noalloc(pr, P.params(tol=1e-4))
    assert st == P.OT_ERR_OOM and "OT_NOALLOC_MAX_BYTES" in P.ot_last_error()
    # unbalanced marginals: invalid, as in ot_solve
    bad = gen.points_sqeuclid(306, 20, 30)
    bad.f = bad.f * 1.01
    pr, _ = P.problem_from_instance(bad, want_plan=False)
    st, _ = P.ot_solve_noalloc(pr, P.params(tol=1e-4))
    assert st == P.OT_ERR_INVALID
