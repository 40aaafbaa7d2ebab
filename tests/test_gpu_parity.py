"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances, and where they come from:
  * Fixed-step trajectories (constant eta, no restarts): the GPU runs the same arithmetic
    as the oracle with a different summation order, so the FP64 plan agrees to a few ulps
    (asserted 1e-13 relative to max|X|).  The FP32 form stores X in FP32 each step: its
    per-entry error stays at the FP32 unit roundoff level (asserted 1e-6 relative).
  * Full adaptive solves: PDHG converges to *an* optimum; X and (u, v) are not unique,
    so the objective, the KKT error and the marginals are compared, never X entrywise.
    At relative KKT tol both the oracle's and the GPU's objective are within a few tol of
    OPT (gap and primal residual are each <= tol), in either direction: at matched
    tol = 1e-6 the objectives are asserted within 5e-6 relative of each other and of the
    exact LP optimum.  The 1e-6 objective bound itself is asserted at matched tol 1e-9
    (FP64 form) and for the FP32 form at tol 1e-7 against the oracle at 1e-9 (its FP32
    storage floor is near 5e-8 in relative KKT).
  * Stored versus regenerated costs use one cost function, so plans are bit-identical.
"""
import json
import os

import numpy as np
import pytest

import oracle
import paper_2407_19689_amd as P
from workloads import generators as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P._abi.load()          # raises if the HIP library is not built
    torch.cuda.set_device(0)


def rel(a, b):
    return abs(a - b) / abs(b)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def run_dense(C, f, g, prec, **kw):
    m, n = C.shape
    X = torch.zeros((m, n), dtype=torch.float64 if prec == P.OT_PREC_FP64 else torch.float32,
                    device="cuda")
    u = torch.zeros(m, dtype=torch.float64, device="cuda")
    v = torch.zeros(n, dtype=torch.float64, device="cuda")
    pr = P.problem(P.OT_COST_DENSE, m, n, dev(f), dev(g), C=dev(C), X_out=X, u_out=u, v_out=v)
    kw.setdefault("time_limit_s", 60.0)
    st, res = P.ot_solve(pr, P.params(precision=prec, **kw))
    torch.cuda.synchronize()
    return st, res.as_dict(), X.double().cpu().numpy(), u.cpu().numpy(), v.cpu().numpy()


def oracle_kkt_bound(prec, gpu_kkt, tol):
    """Bound for the oracle's relative KKT of a returned triple.  The FP64 form uses the
    oracle's costs: its verified KKT (<= tol) is confirmed up to summation order.  The FP32
    form is verified against its FP32-rounded costs (each within 2^-24 relative of the FP64
    cost, and C >= 0): that moves rel_D by at most 2^-24 (||dC|| <= 2^-24 ||C||) and rel_G
    by at most 2^-24 (|<dC, X>| <= 2^-24 <C, X>), so the oracle's value is within
    sqrt(2) * 2^-24 of the GPU's."""
    if prec == P.OT_PREC_FP64:
        return tol * (1 + 1e-6)
    return gpu_kkt * (1 + 1e-6) + np.sqrt(2.0) * 2.0 ** -24


def random_problem(seed, m, n):
    rng = np.random.default_rng(seed)
    C = rng.uniform(size=(m, n))
    f = rng.uniform(0.1, 1, m)
    f /= f.sum()
    g = rng.uniform(0.1, 1, n)
    g /= g.sum()
    return C, f, g


# ----------------------------------------------------------- fixed-step trajectory parity

SHAPES = [(37, 203, 1, 16), (37, 203, 2, 32), (37, 203, 4, 16), (1, 5, 1, 16), (9, 1, 1, 16),
          (300, 517, 4, 64), (130, 70, 2, 48), (64, 64, 4, 16)]


# engine 1: every slot one launch over the whole GPU; engine 2: one work-group runs the
# whole instance (resident)
ENGINES = [1, 2]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
@pytest.mark.parametrize("m,n,vec,rows", SHAPES)
def test_fixed_step_trajectory_matches_oracle(prec, m, n, vec, rows, engine):
    """Algorithm 2 with a constant step and no restart: the GPU's 30th iterate equals the
    oracle's (current iterate returned, output = 1)."""
    C, f, g = random_problem(m * 1000 + n, m, n)
    K, eta, omega = 30, 0.5 / np.sqrt(m + n), 1.3
    common = dict(tol=1e-12, max_iters=K, step_rule=1, restart_rule=2, output=1, eta0=eta,
                  omega0=omega)
    Xo, po, qo, ro, _ = oracle.solve(C, f, g, **common)
    st, res, X, u, v = run_dense(C, f, g, prec, tile_vec=vec, tile_rows=rows, engine=engine,
                                 **common)
    assert st == P.OT_NOT_CONVERGED and res["iterations"] == K
    scale = np.abs(Xo).max()
    lim = 1e-13 if prec == P.OT_PREC_FP64 else 1e-6
    assert np.abs(X - Xo).max() <= lim * scale
    dual_scale = max(np.abs(po).max(), np.abs(qo).max())
    assert np.abs(u - po).max() <= lim * dual_scale * 10
    assert np.abs(v - qo).max() <= lim * dual_scale * 10


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
@pytest.mark.parametrize("omega,iters,avg", [(0.8, 25, 0), (10.0, 24, 1), (10.0, 25, 1)])
def test_average_and_candidate_match_oracle(prec, engine, omega, iters, avg):
    """With output = 0 the returned plan is the restart candidate: the running average when
    its KKT error is not larger (Section 5).  Same candidate and same average as the
    oracle (fixed step, no restart).  The stored average lags by one iterate after an odd
    number of accepted steps, so an average returned after 25 iterations goes through a
    fold pass and one returned after 24 does not."""
    C, f, g = random_problem(7, 45, 77)
    common = dict(tol=1e-12, max_iters=iters, step_rule=1, restart_rule=2, output=0,
                  eta0=0.6 / np.sqrt(122), omega0=omega)
    Xo, po, qo, ro, _ = oracle.solve(C, f, g, **common)
    st, res, X, u, v = run_dense(C, f, g, prec, engine=engine, **common)
    assert res["returned_average"] == ro["returned_average"] == avg
    assert res["mode_passes"][6] == avg * (iters % 2)
    lim = 1e-13 if prec == P.OT_PREC_FP64 else 1e-6
    assert np.abs(X - Xo).max() <= lim * np.abs(Xo).max()
    assert np.abs(u - po).max() <= lim * np.abs(po).max() * 10


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
def test_restarts_to_the_average_match_oracle(prec, engine):
    """Fixed step with the adaptive restarts of Section 5 for 300 iterations: the same
    restarts as the oracle, and the same final iterate.  Some restarts go to an average
    that does not yet hold the current iterate (a fold pass runs first)."""
    C, f, g = random_problem(11, 45, 77)
    common = dict(tol=1e-12, max_iters=300, step_rule=1, restart_rule=0, output=1,
                  eta0=0.6 / np.sqrt(122), omega0=0.8)
    Xo, po, qo, ro, _ = oracle.solve(C, f, g, **common)
    st, res, X, u, v = run_dense(C, f, g, prec, engine=engine, **common)
    assert st == P.OT_NOT_CONVERGED and res["iterations"] == 300
    if prec == P.OT_PREC_FP64:
        assert res["restarts"] == ro["restarts"] > 0
        assert np.abs(X - Xo).max() <= 1e-10 * np.abs(Xo).max()
    assert res["mode_passes"][6] >= 1


# ----------------------------------------------------------- full adaptive solves

def highs_opt(C, f, g):
    from scipy.optimize import linprog
    from scipy.sparse import csr_matrix
    m, n = C.shape
    rows, cols = [], []
    for i in range(m):
        for j in range(n):
            rows += [i, m + j]
            cols += [i * n + j, i * n + j]
    A = csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(m + n, m * n))
    r = linprog(C.reshape(-1), A_eq=A, b_eq=np.concatenate([f, g]), bounds=(0, None),
                method="highs")
    assert r.status == 0
    return r.fun


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
def test_config1_solve_matches_oracle_and_exact_lp(seed, prec, engine):
    inst = gen.config_instance(1, seed)
    C = inst.dense_cost()
    _, _, _, ref, _ = oracle.solve(C, inst.f, inst.g, tol=1e-6)
    opt = highs_opt(C, inst.f, inst.g)
    st, res, out = P.solve_instance(inst, P.params(tol=1e-6, precision=prec, engine=engine,
                                                   time_limit_s=60.0))
    torch.cuda.synchronize()
    assert st == P.OT_OK, P.ot_last_error()
    assert res["rel_kkt"] <= 1e-6
    X = out["X"].double().cpu().numpy()
    k = oracle.kkt(C, inst.f, inst.g, X, out["u"].cpu().numpy(), out["v"].cpu().numpy())
    assert k["rel_kkt"] <= oracle_kkt_bound(prec, res["rel_kkt"], 1e-6)   # the oracle confirms it
    # the FP32 form's objective uses its FP32 cost entries (each within 2^-24 relative of
    # the FP64 cost the oracle uses); the FP64 form uses the same cost as the oracle
    lim = 1e-12 if prec == P.OT_PREC_FP64 else 2.0 ** -24
    assert rel(k["objective"], res["objective"]) <= lim
    assert rel(res["objective"], ref["objective"]) <= 5e-6
    assert rel(res["objective"], opt) <= 5e-6
    assert np.all(X >= 0)


@pytest.mark.parametrize("prec,tol", [(P.OT_PREC_FP64, 1e-9), (P.OT_PREC_FP32, 1e-7)])
def test_objective_within_1e6_of_oracle_at_tight_tolerance(prec, tol):
    for seed in range(3):
        inst = gen.config_instance(1, seed)
        C = inst.dense_cost()
        _, _, _, ref, _ = oracle.solve(C, inst.f, inst.g, tol=1e-9, max_iters=400000)
        st, res, _ = P.solve_instance(inst, P.params(tol=tol, precision=prec, time_limit_s=60.0))
        assert st == P.OT_OK, P.ot_last_error()
        assert res["rel_kkt"] <= tol
        assert rel(res["objective"], ref["objective"]) <= 1e-6


def assert_matches_oracle(inst, res, out, prec, solve_limit=200_000):
    """A result from a batch or the server against the oracle: the oracle recomputes the
    KKT error of the returned triple (it meets the tolerance) and its certified bracket;
    for instances of at most solve_limit plan entries (the oracle's own solve takes seconds
    there) the objective also agrees with the oracle's solve at the same tolerance, within
    the sum of the two results' certified bracket widths (both brackets contain OPT) and
    within 5 tol."""
    C = inst.dense_cost()
    tol = inst.tol
    X = out["X"].double().cpu().numpy()
    u = out["u"].cpu().numpy()
    k = oracle.kkt(C, inst.f, inst.g, X, u, out["v"].cpu().numpy())
    assert res["status"] == P.OT_OK and res["rel_kkt"] <= tol
    assert k["rel_kkt"] <= oracle_kkt_bound(prec, res["rel_kkt"], tol)
    lb_g, ub_g = certified_bracket(C, inst.f, inst.g, X, u)
    assert lb_g - 5 * tol * abs(res["objective"]) <= res["objective"]
    assert res["objective"] <= ub_g + 5 * tol * abs(res["objective"])
    if inst.m * inst.n > solve_limit:
        return
    Xo, po, _, ro, _ = oracle.solve(C, inst.f, inst.g, tol=tol, max_iters=400000)
    assert ro["status"] == 0
    lb_o, ub_o = certified_bracket(C, inst.f, inst.g, Xo, po)
    assert max(lb_g, lb_o) <= min(ub_g, ub_o) * (1 + 1e-12)    # both contain OPT
    # each objective is within the farther end of its own bracket from OPT
    dist_g = max(ub_g - res["objective"], res["objective"] - lb_g)
    dist_o = max(ub_o - ro["objective"], ro["objective"] - lb_o)
    assert abs(res["objective"] - ro["objective"]) <= dist_g + dist_o + 1e-15
    assert rel(res["objective"], ro["objective"]) <= 5 * tol


def golden(name):
    with open(os.path.join(HERE, "golden", name)) as fh:
        return json.load(fh)


def certified_bracket(C, f, g, X, u):
    """[lower, upper] around OPT from any returned triple, by the oracle: the c-transform
    of u gives a dual-feasible pair (weak duality, lower) and Algorithm 3 an exactly
    feasible plan near X (its cost, upper)."""
    lb = oracle.dual_lower_bound(C, f, g, u)
    ub = float((C * oracle.round_plan(f, g, X)).sum())
    assert lb <= ub * (1 + 1e-12)
    return lb, ub


def assert_objective_at_tol(C, f, g, res, X, u, opt_ref, ref_tol):
    """At a relative KKT tolerance the objective of a triple is determined only up to the
    distance its own certified bracket allows: OPT lies in [lb, ub], and so does the
    oracle's tight-tolerance objective (to ref_tol), so
        |obj - opt_ref| <= max(ub - obj, obj - lb) + ref_tol * |opt_ref|.
    Returns that bound relative to opt_ref."""
    lb, ub = certified_bracket(C, f, g, X, u)
    obj = res["objective"]
    assert lb * (1 - 1e-12) <= opt_ref * (1 + 2 * ref_tol)
    assert opt_ref * (1 - 2 * ref_tol) <= ub * (1 + 1e-12)
    bound = max(ub - obj, obj - lb, 0.0) + ref_tol * abs(opt_ref)
    assert abs(obj - opt_ref) <= bound
    return bound / abs(opt_ref)


@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
def test_config2_grid_1024_matches_oracle(prec):
    """m = n = 1024 (32x32 blob images, squared pixel cost regenerated on the GPU); the
    oracle's objectives at tol 1e-6 and 1e-9 are stored in tests/golden (written by
    tests/golden/make_golden.py, which calls only the oracle).  At matched tol 1e-6 the
    objective is within the distance its certified bracket allows of the oracle's tol-1e-9
    objective (and that distance is a few 1e-6 at most); at a tight tolerance (FP64 1e-9,
    FP32 1e-7, above its storage floor) it is within 1e-6."""
    gold = golden("config2_oracle.json")
    inst = gen.config_instance(2, 0)
    C = inst.dense_cost()
    opt = gold["objective_tol1e-09"]
    st, res, out = P.solve_instance(inst, P.params(tol=1e-6, precision=prec, time_limit_s=60.0))
    assert st == P.OT_OK, P.ot_last_error()
    assert res["rel_kkt"] <= 1e-6
    b = assert_objective_at_tol(C, inst.f, inst.g, res, out["X"].double().cpu().numpy(),
                                out["u"].cpu().numpy(), opt, 1e-9)
    assert b <= 2e-5
    assert rel(res["objective"], gold["objective_tol1e-06"]) <= 5e-6
    tight = 1e-9 if prec == P.OT_PREC_FP64 else 1e-7
    st, res, _ = P.solve_instance(inst, P.params(tol=tight, precision=prec, time_limit_s=60.0))
    assert st == P.OT_OK, P.ot_last_error()
    assert res["rel_kkt"] <= tight
    assert rel(res["objective"], opt) <= 1e-6


@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
def test_config3_grid_4096_objective_matches_oracle(prec):
    """The benchmark instance (m = n = 4096, 64x64 blob images, cost regenerated in the
    kernel) against the oracle's objective at tol 1e-8 (tests/golden/config3_oracle.json,
    oracle only): within 1e-6 when solved to a tight tolerance (FP64 1e-8, FP32 1e-7), and
    at matched tol 1e-6 within the distance the result's own certified bracket allows."""
    gold = golden("config3_oracle.json")
    inst = gen.config_instance(3, 0)
    C = inst.dense_cost()
    opt = gold["objective_tol1e-08"]
    assert gold["lower_tol1e-08"] <= opt <= gold["upper_tol1e-08"]
    tight = 1e-8 if prec == P.OT_PREC_FP64 else 1e-7
    st, res, _ = P.solve_instance(inst, P.params(tol=tight, precision=prec, time_limit_s=120.0))
    assert st == P.OT_OK, P.ot_last_error()
    assert res["rel_kkt"] <= tight
    assert rel(res["objective"], opt) <= 1e-6
    st, res, out = P.solve_instance(inst, P.params(tol=1e-6, precision=prec, time_limit_s=120.0))
    assert st == P.OT_OK, P.ot_last_error()
    b = assert_objective_at_tol(C, inst.f, inst.g, res, out["X"].double().cpu().numpy(),
                                out["u"].cpu().numpy(), opt, 1e-8)
    assert b <= 2e-5


def test_config3_grid_4096_verified_and_bracketed():
    """Full size of the benchmark (m = n = 4096, FP32 plan, cost regenerated in-kernel):
    the oracle recomputes the KKT error of the returned triple, and the objective lies in
    the certified bracket [f.u + g.v^c, <C, round(X)>] (weak duality with the c-transform;
    Algorithm 3 gives an exactly feasible plan) widened by the tolerance."""
    inst = gen.config_instance(3, 0)
    st, res, out = P.solve_instance(inst, P.params(tol=1e-6, precision=P.OT_PREC_FP32,
                                                   time_limit_s=120.0))
    assert st == P.OT_OK, P.ot_last_error()
    X = out["X"].double().cpu().numpy()
    u = out["u"].cpu().numpy()
    v = out["v"].cpu().numpy()
    C = inst.dense_cost()
    k = oracle.kkt(C, inst.f, inst.g, X, u, v)
    assert k["rel_kkt"] <= oracle_kkt_bound(P.OT_PREC_FP32, res["rel_kkt"], 1e-6)
    lb, ub = certified_bracket(C, inst.f, inst.g, X, u)
    obj = res["objective"]
    assert lb - 5e-6 * obj <= obj <= ub + 5e-6 * obj
    assert (ub - lb) / obj <= 2e-5
    # the GPU's rounding and bracket of the same plan agree with the oracle's
    pr, _ = P.problem_from_instance(inst, want_plan=False)
    st, br = P.ot_round(pr, P.OT_PREC_FP32, out["X"], out["u"])
    assert st == P.OT_OK, P.ot_last_error()
    assert rel(br["lower"], lb) <= 1e-11 and rel(br["upper"], ub) <= 1e-11
    assert br["feas_violation"] <= 1e-15


# ----------------------------------------------------------- cost sources

@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
@pytest.mark.parametrize("which", ["grid", "points_sq", "points_eu", "grid_l1", "grid_l2",
                                   "grid_linf"])
def test_stored_and_regenerated_costs_give_identical_plans(prec, which, engine):
    if which == "grid":
        inst = gen.grid_pair(5, 12, tol=1e-6)
    elif which.startswith("grid_"):
        inst = gen.grid_pair(5, 11, kind=which, tol=1e-6)
    elif which == "points_sq":
        inst = gen.points_sqeuclid(5, 90, 300, tol=1e-6)
    else:
        inst = gen.gmm_euclid(5, 120, 70, tol=1e-6)
    outs = []
    for store in (0, 1):
        st, res, out = P.solve_instance(inst, P.params(tol=1e-6, precision=prec, engine=engine,
                                                       time_limit_s=60.0), store=store)
        assert st == P.OT_OK, P.ot_last_error()
        outs.append((res, out["X"].cpu().numpy()))
    assert outs[0][0]["iterations"] == outs[1][0]["iterations"]
    assert np.array_equal(outs[0][1], outs[1][1])


def test_fp64_regenerated_cost_equals_dense_oracle_cost():
    """The FP64 kernel's cost equals numpy's FP64 cost bit for bit (no contraction), so the
    dense and regenerated FP64 solves follow the same trajectory."""
    for inst in (gen.points_sqeuclid(3, 50, 70), gen.grid_pair(3, 10), gen.gmm_euclid(3, 40, 33),
                 gen.grid_pair(3, 9, kind="grid_l1"), gen.grid_pair(3, 9, kind="grid_l2"),
                 gen.grid_pair(3, 9, kind="grid_linf")):
        a = P.solve_instance(inst, P.params(tol=1e-6, precision=P.OT_PREC_FP64), dense=True)
        b = P.solve_instance(inst, P.params(tol=1e-6, precision=P.OT_PREC_FP64), dense=False)
        assert a[1]["iterations"] == b[1]["iterations"]
        assert np.array_equal(a[2]["X"].cpu().numpy(), b[2]["X"].cpu().numpy())


@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
@pytest.mark.parametrize("kind", ["grid_l1", "grid_l2", "grid_linf"])
def test_grid_norm_costs_match_oracle(prec, kind):
    """The l1, l2 and l-infinity pixel costs of Section 5.1, regenerated in the kernel:
    the oracle (dense FP64 cost) confirms the KKT error of the returned triple, and the
    objective agrees with the oracle's at the same tolerance and with the exact optimum."""
    inst = gen.grid_pair(17, 12, kind=kind, tol=1e-6)
    C = inst.dense_cost()
    _, _, _, ref, _ = oracle.solve(C, inst.f, inst.g, tol=1e-6, max_iters=400000)
    opt = highs_opt(C, inst.f, inst.g)
    st, res, out = P.solve_instance(inst, P.params(tol=1e-6, precision=prec, time_limit_s=60.0))
    assert st == P.OT_OK, P.ot_last_error()
    k = oracle.kkt(C, inst.f, inst.g, out["X"].double().cpu().numpy(), out["u"].cpu().numpy(),
                   out["v"].cpu().numpy())
    assert k["rel_kkt"] <= oracle_kkt_bound(prec, res["rel_kkt"], 1e-6)
    assert rel(res["objective"], ref["objective"]) <= 5e-6
    assert rel(res["objective"], opt) <= 5e-6


@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
def test_paper_literal_mode_matches_oracle(prec):
    """Algorithm 2 as printed: constant step eta = 1/(2 ||A||_2) = 1/(2 sqrt(m+n)) (the
    theory's step), uniform averaging, the basic restart condition KKT(average) <=
    beta KKT(restart point) with a restart to the average, fixed primal weight.  The oracle
    in the same mode: the GPU's returned triple passes the oracle's KKT check, its objective
    agrees, and in FP64 the two take the same number of iterations up to a few percent
    (decisions compare KKT values computed with different summation orders; the FP32 form
    rounds the plan every step and follows its own path)."""
    inst = gen.config_instance(1, 2)
    C = inst.dense_cost()
    mode = dict(tol=1e-5, step_rule=1, restart_rule=1, avg_weighting=1, primal_weight_update=0,
                eta0=0.5 / np.sqrt(inst.m + inst.n), beta_basic=0.2, max_iters=400000)
    _, _, _, ref, _ = oracle.solve(C, inst.f, inst.g, **mode)
    st, res, out = P.solve_instance(inst, P.params(precision=prec, time_limit_s=120.0, **mode))
    assert st == P.OT_OK, P.ot_last_error()
    k = oracle.kkt(C, inst.f, inst.g, out["X"].double().cpu().numpy(), out["u"].cpu().numpy(),
                   out["v"].cpu().numpy())
    assert k["rel_kkt"] <= oracle_kkt_bound(prec, res["rel_kkt"], 1e-5)
    assert rel(res["objective"], ref["objective"]) <= 5e-5
    assert res["restarts"] >= 1 and ref["restarts"] >= 1
    if prec == P.OT_PREC_FP64:
        assert abs(res["iterations"] - ref["iterations"]) <= 0.05 * ref["iterations"] + 2


# ----------------------------------------------------------- degenerate cases

@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
def test_single_row_and_single_column_plans_are_forced(prec):
    """m = 1 or n = 1: the plan is forced.  The FP64 form reaches tol 1e-8; the FP32 form
    stores the plan in FP32 (relative KKT floor near 5e-8), so below its floor (1e-8) its
    returned arrays fail the final verification and, once its retries are used up, the solve
    reports OT_NOT_CONVERGED with its outputs filled, never OT_OK; at every tolerance a
    solve reports OT_OK exactly when its verified relative KKT meets the tolerance."""
    rng = np.random.default_rng(9)
    n = 37
    C = rng.uniform(size=(1, n))
    g = rng.uniform(0.1, 1, n)
    g /= g.sum()
    tols = (1e-8,) if prec == P.OT_PREC_FP64 else (1e-8, 1e-7)
    for tol in tols:
        for Cc, f1, g1, axis in ((C, np.array([1.0]), g, 0), (C.T.copy(), g, np.array([1.0]), 1)):
            st, res, X, u, v = run_dense(Cc, f1, g1, prec, tol=tol)
            assert st in (P.OT_OK, P.OT_NOT_CONVERGED), (tol, st)
            assert (res["rel_kkt"] <= tol) == (st == P.OT_OK), (tol, st, res["rel_kkt"])
            if prec == P.OT_PREC_FP64:
                assert st == P.OT_OK
            if prec == P.OT_PREC_FP32 and tol == 1e-8:
                assert st == P.OT_NOT_CONVERGED and res["verify_retries"] == 8
            np.testing.assert_allclose(X[0] if axis == 0 else X[:, 0], g, atol=2e-7)


def test_separable_cost_and_zero_cost():
    rng = np.random.default_rng(10)
    m, n = 33, 71
    a, b = rng.uniform(size=m), rng.uniform(size=n)
    _, f, g = random_problem(11, m, n)
    st, res, X, u, v = run_dense(a[:, None] + b[None, :], f, g, P.OT_PREC_FP64, tol=1e-9)
    assert st == P.OT_OK
    assert rel(res["objective"], a @ f + b @ g) <= 1e-8
    # C = 0: the start point X = 0 is infeasible; every feasible plan is optimal with OPT 0.
    # With OPT = 0 the scale-free relative gap |pobj - dobj| / (|pobj| + |dobj|) stays at 1
    # for any dobj != 0, so this case uses the 1 + scale denominators (kkt_mode 1).
    st, res, X, u, v = run_dense(np.zeros((m, n)), f, g, P.OT_PREC_FP64, tol=1e-8, kkt_mode=1)
    assert st == P.OT_OK
    assert abs(res["objective"]) == 0.0
    assert res["rel_primal"] <= 1e-8


def test_identical_marginals_on_a_metric_cost_have_zero_optimum():
    inst = gen.grid_pair(21, 9)
    C = inst.dense_cost()
    # OPT = 0: the relative gap needs the 1 + scale denominators (see the zero-cost case)
    st, res, X, u, v = run_dense(C, inst.f, inst.f.copy(), P.OT_PREC_FP64, tol=1e-8, kkt_mode=1)
    assert st == P.OT_OK
    assert res["objective"] <= 1e-7 * C.max()


# ----------------------------------------------------------- failure paths

def test_nonfinite_cost_is_reported_numeric():
    C, f, g = random_problem(3, 20, 30)
    C[4, 7] = np.nan
    st, res, X, u, v = run_dense(C, f, g, P.OT_PREC_FP64)
    assert st == P.OT_ERR_NUMERIC


def test_iteration_limit_returns_filled_outputs():
    C, f, g = random_problem(4, 40, 50)
    st, res, X, u, v = run_dense(C, f, g, P.OT_PREC_FP32, tol=1e-9, max_iters=5)
    assert st == P.OT_NOT_CONVERGED
    assert res["iterations"] == 5 and res["rel_kkt"] > 1e-9
    assert np.all(np.isfinite(X)) and np.all(np.isfinite(u)) and np.all(np.isfinite(v))
    k = oracle.kkt(C, f, g, X, u, v)
    assert rel(k["rel_kkt"], res["rel_kkt"]) <= 1e-9


def test_time_limit_stops_the_solve():
    inst = gen.grid_pair(3, 48)
    st, res, _ = P.solve_instance(inst, P.params(tol=1e-12, time_limit_s=0.05, graph_slots=16))
    assert st == P.OT_NOT_CONVERGED
    assert res["seconds"] < 5.0


def test_unbalanced_or_negative_marginals_are_invalid():
    C, f, g = random_problem(5, 10, 12)
    st, *_ = run_dense(C, f * 1.001, g, P.OT_PREC_FP64)
    assert st == P.OT_ERR_INVALID
    f2 = f.copy()
    f2[0] = -f2[0]
    g2 = g * (f2.sum() / g.sum())
    st, *_ = run_dense(C, f2, g2, P.OT_PREC_FP64)
    assert st == P.OT_ERR_INVALID


# ----------------------------------------------------------- determinism, batch, plumbing

@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
def test_resident_and_grid_engines_agree(prec):
    """The two execution paths run the same method with different summation orders: both
    meet the tolerance (confirmed by the oracle's KKT) and their objectives agree to the
    accuracy the tolerance fixes; each path is deterministic."""
    for inst in (gen.points_sqeuclid(31, 120, 200, tol=1e-6), gen.grid_pair(32, 11, tol=1e-6),
                 gen.gmm_euclid(33, 250, 90, tol=1e-6)):
        C = inst.dense_cost()
        objs = []
        for engine in ENGINES:
            prm = P.params(tol=1e-6, precision=prec, engine=engine, time_limit_s=60.0)
            st, res, out = P.solve_instance(inst, prm)
            assert st == P.OT_OK, P.ot_last_error()
            k = oracle.kkt(C, inst.f, inst.g, out["X"].double().cpu().numpy(),
                           out["u"].cpu().numpy(), out["v"].cpu().numpy())
            assert k["rel_kkt"] <= oracle_kkt_bound(prec, res["rel_kkt"], 1e-6)
            st2, res2, out2 = P.solve_instance(inst, prm)
            assert res2["iterations"] == res["iterations"]
            assert np.array_equal(out2["X"].cpu().numpy(), out["X"].cpu().numpy())
            objs.append(res["objective"])
        assert rel(objs[0], objs[1]) <= 5e-6


def test_resident_instances_beside_grid_instances_in_one_batch():
    """A batch whose instances straddle the resident threshold: the resident ones run on
    their own stream beside the graph of the others, and every result equals its solo
    solve."""
    insts = [gen.points_sqeuclid(60 + i, m, n, tol=1e-5)
             for i, (m, n) in enumerate([(64, 64), (300, 300), (180, 360), (700, 650), (20, 3000)])]
    prm = P.params(tol=1e-5, precision=P.OT_PREC_FP32, time_limit_s=60.0)
    probs, outs = [], []
    for inst in insts:
        pr, out = P.problem_from_instance(inst, tol=inst.tol)
        probs.append(pr)
        outs.append(out)
    st, results = P.ot_solve_batch(probs, prm)
    torch.cuda.synchronize()
    assert st == P.OT_OK, P.ot_last_error()
    for inst, out, rb in zip(insts, outs, results):
        s1, r1, o1 = P.solve_instance(inst, prm, tol=inst.tol)
        assert s1 == P.OT_OK
        assert rb.iterations == r1["iterations"]
        assert np.array_equal(out["X"].cpu().numpy(), o1["X"].cpu().numpy())
        assert_matches_oracle(inst, rb.as_dict(), out, P.OT_PREC_FP32)


# ----------------------------------------------------------- rounding and bracket

@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
@pytest.mark.parametrize("which", ["dense", "grid", "points_eu"])
def test_rounding_and_bracket_match_oracle(prec, which):
    """Algorithm 3 on the GPU equals the oracle's rounding of the same plan (FP64, different
    summation order), the bracket equals the oracle's weak-duality bound and the cost of the
    rounded plan, the rounded plan is feasible to rounding error, and Lemma lem:round's
    bound on the change holds."""
    if which == "dense":
        C, f, g = random_problem(21, 70, 130)
        inst = None
    elif which == "grid":
        inst = gen.grid_pair(22, 12, tol=1e-4)
    else:
        inst = gen.gmm_euclid(23, 150, 90, tol=1e-4)
    prm = P.params(tol=1e-4, precision=prec, time_limit_s=60.0)
    if inst is None:
        st, res, X, u, v = run_dense(C, f, g, prec, tol=1e-4)
        pr = P.problem(P.OT_COST_DENSE, 70, 130, dev(f), dev(g), C=dev(C))
        Xin = X.astype(np.float32) if prec == P.OT_PREC_FP32 else X
    else:
        C, f, g = inst.dense_cost(), inst.f, inst.g
        st, res, out = P.solve_instance(inst, prm)
        X = out["X"].double().cpu().numpy()
        u = out["u"].cpu().numpy()
        pr, _ = P.problem_from_instance(inst, want_plan=False)
        Xin = out["X"].cpu().numpy()
    assert st == P.OT_OK, P.ot_last_error()
    Xf = np.empty_like(X)
    st, br = P.ot_round(pr, prec, Xin, u, X_feas=Xf)
    assert st == P.OT_OK, P.ot_last_error()
    ref = oracle.round_plan(f, g, X)
    assert np.abs(Xf - ref).max() <= 1e-13 * np.abs(ref).max()
    # err_r, err_c >= 0 in exact arithmetic; in FP64 an err_c_j can be a few ulps below 0
    # where the scaled plan is 0, so entries are nonnegative up to rounding (as the oracle's)
    assert Xf.min() >= -1e-14 * Xf.max()
    lb = oracle.dual_lower_bound(C, f, g, u)
    assert rel(br["lower"], lb) <= 1e-12
    assert rel(br["upper"], float((C * ref).sum())) <= 1e-12
    assert br["lower"] <= br["upper"]
    assert br["feas_violation"] <= 1e-15
    assert abs(Xf.sum(axis=1) - f).max() <= 1e-15 and abs(Xf.sum(axis=0) - g).max() <= 1e-15
    marg = np.abs(f - X.sum(axis=1)).sum() + np.abs(g - X.sum(axis=0)).sum()
    assert rel(br["marginal_l1"], marg) <= 1e-9
    assert br["l1_change"] <= 2.0 * br["marginal_l1"] * (1 + 1e-12)
    # the bracket contains the exact optimum
    opt = highs_opt(C, f, g)
    assert br["lower"] <= opt * (1 + 1e-12) and opt <= br["upper"] * (1 + 1e-12)


def test_repeated_solves_are_bit_identical():
    inst = gen.grid_pair(8, 40)
    a = P.solve_instance(inst, P.params(tol=1e-5))
    b = P.solve_instance(inst, P.params(tol=1e-5))
    assert a[1]["iterations"] == b[1]["iterations"]
    assert np.array_equal(a[2]["X"].cpu().numpy(), b[2]["X"].cpu().numpy())
    assert np.array_equal(a[2]["u"].cpu().numpy(), b[2]["u"].cpu().numpy())


@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
def test_profile_mode_solves_like_graph_mode_and_times_every_pass(prec):
    # profile mode launches the same kernels without a graph: identical iterates, and the
    # event-timed launches are those of the solve (counted by kind, fold passes included)
    inst = gen.grid_pair(46, 32, tol=1e-6)
    a = P.solve_instance(inst, P.params(tol=1e-6, precision=prec))
    b = P.solve_instance(inst, P.params(tol=1e-6, precision=prec, profile=1))
    assert a[0] == P.OT_OK and b[0] == P.OT_OK
    assert a[1]["iterations"] == b[1]["iterations"] and a[1]["restarts"] == b[1]["restarts"]
    assert np.array_equal(a[2]["X"].cpu().numpy(), b[2]["X"].cpu().numpy())
    r = b[1]
    assert sum(r["mode_passes"]) == r["kernel_passes"]
    assert r["pass_ms"] > 0.0 and r["combine_ms"] > 0.0
    # each timed pass lasts at least a microsecond and on average well under a millisecond
    assert 1e-3 * r["kernel_passes"] < r["pass_ms"] < 1.0 * r["kernel_passes"]
    # passes that fold two iterates are trial or full passes, about every other one
    full_trial = r["mode_passes"][2] + r["mode_passes"][3]
    assert 0.3 * full_trial < r["avg_fold_passes"] <= full_trial


@pytest.mark.parametrize("prec", [P.OT_PREC_FP64, P.OT_PREC_FP32])
def test_batch_equals_solo(prec):
    insts = [gen.gmm_euclid(40 + i, m, n, tol=1e-5)
             for i, (m, n) in enumerate([(33, 700), (512, 48), (260, 260), (1, 90), (97, 1)])]
    insts.append(gen.grid_pair(45, 14, tol=1e-5))
    prm = P.params(tol=1e-5, precision=prec, time_limit_s=60.0)
    probs, outs = [], []
    for inst in insts:
        pr, out = P.problem_from_instance(inst, precision=prec, tol=inst.tol)
        probs.append(pr)
        outs.append(out)
    st, results = P.ot_solve_batch(probs, prm)
    torch.cuda.synchronize()
    assert st == P.OT_OK, P.ot_last_error()
    for inst, out, rb in zip(insts, outs, results):
        s1, r1, o1 = P.solve_instance(inst, prm, tol=inst.tol)
        assert s1 == P.OT_OK
        assert rb.iterations == r1["iterations"] and rb.restarts == r1["restarts"]
        assert np.array_equal(out["X"].cpu().numpy(), o1["X"].cpu().numpy())
        assert np.array_equal(out["u"].cpu().numpy(), o1["u"].cpu().numpy())
        assert_matches_oracle(inst, rb.as_dict(), out, prec)


def test_caller_workspace_and_stream():
    inst = gen.points_sqeuclid(12, 200, 150, tol=1e-6)
    prm = P.params(tol=1e-6)
    pr, out = P.problem_from_instance(inst)
    nbytes = P.ot_workspace_size(pr, prm)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    st, res = P.ot_solve(pr, prm, workspace=ws, stream=stream.cuda_stream)
    assert st == P.OT_OK
    s2, r2, o2 = P.solve_instance(inst, prm)
    assert res.iterations == r2["iterations"]
    assert np.array_equal(out["X"].cpu().numpy(), o2["X"].cpu().numpy())
    small = torch.empty(nbytes // 2, dtype=torch.uint8, device="cuda")
    st, _ = P.ot_solve(pr, prm, workspace=small)
    assert st == P.OT_ERR_OOM


@pytest.mark.parametrize("prec", [P.OT_PREC_FP32, P.OT_PREC_FP64])
def test_write_through_plan_stores_change_no_value(prec):
    """A solve whose plans fit 8 MB stores them through L2 (agent-scope stores); the same
    1024 x 1024 instance solved in a batch beside a 2304 x 2304 one (plans over the limit,
    ordinary stores) gives the same iterates bit for bit, and both match the oracle."""
    small = gen.grid_pair(46, 32, tol=1e-5)
    big = gen.grid_pair(47, 48, tol=1e-4)
    prm = P.params(tol=1e-5, precision=prec, time_limit_s=60.0)
    s1, r1, o1 = P.solve_instance(small, prm, tol=small.tol)
    assert s1 == P.OT_OK
    probs, outs = [], []
    for inst in (small, big):
        pr, out = P.problem_from_instance(inst, precision=prec, tol=inst.tol)
        probs.append(pr)
        outs.append(out)
    st, results = P.ot_solve_batch(probs, prm)
    torch.cuda.synchronize()
    assert st == P.OT_OK, P.ot_last_error()
    assert results[0].iterations == r1["iterations"]
    assert np.array_equal(outs[0]["X"].cpu().numpy(), o1["X"].cpu().numpy())
    assert np.array_equal(outs[0]["u"].cpu().numpy(), o1["u"].cpu().numpy())
    assert np.array_equal(outs[0]["v"].cpu().numpy(), o1["v"].cpu().numpy())
    assert_matches_oracle(small, r1, o1, prec)
