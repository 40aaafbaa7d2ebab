"""Pins of the FP64 oracle against facts fixed by the paper or by mathematics.

Each test checks the oracle against something other than itself:
  * Algorithm 1 on the explicit Kronecker matrix A (Section 3.1) -- the paper states its
    iterates equal Algorithm 2's under vec (Section 4.1, equivalence of iterates);
  * the adjoint/Kronecker identities of the matrix-free products (Section 3.1);
  * ||A||_2 = sqrt(m+n) (Proposition prop:norm-sharp, attained at the all-ones vector);
  * exact optima from independent textbook solvers (tests/exact_lp.py) and HiGHS;
  * invariants: sum p = sum q from a zero start, cost shift, transposition, exact
    power-of-two scaling (the scaled-LP identity of Section 4.2);
  * closed forms inside the control: constant-eta averaging is the arithmetic mean
    (Algorithm 2), theta = 1/2 primal weight is a geometric mean (Section 5);
  * the rounding lemma (lem:round) and weak duality for the certified bracket.
"""
import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.sparse import csr_matrix

from tests import exact_lp
from workloads import generators as gen


def kron_A(m, n):
    """A = [1_n^T kron I_m ; I_n kron 1_m^T] acting on column-major vec(X)."""
    return np.vstack([np.kron(np.ones((1, n)), np.eye(m)), np.kron(np.eye(n), np.ones((1, m)))])


def vec(X):
    return X.reshape(-1, order="F")


def random_instance(rng, m, n, kind="uniform"):
    C = rng.uniform(0.0, 1.0, size=(m, n))
    f = rng.uniform(0.1, 1.0, size=m)
    g = rng.uniform(0.1, 1.0, size=n)
    f /= f.sum()
    g /= g.sum()
    g *= f.sum() / g.sum()
    return C, f, g


def highs_opt(C, f, g):
    m, n = C.shape
    rows, cols = [], []
    for i in range(m):
        for j in range(n):
            rows += [i, m + j]
            cols += [i * n + j, i * n + j]
    A = csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(m + n, m * n))
    res = linprog(C.reshape(-1), A_eq=A, b_eq=np.concatenate([f, g]), bounds=(0, None),
                  method="highs")
    assert res.status == 0
    return res.fun, res


# ---------------------------------------------------------------- P-1, P-7 (averaging)

@pytest.mark.parametrize("m,n", [(5, 7), (9, 4), (1, 6)])
def test_algorithm1_on_explicit_A_equals_oracle(orc, m, n):
    rng = np.random.default_rng(11 + m * n)
    C, f, g = random_instance(rng, m, n)
    A = kron_A(m, n)
    c, b = vec(C), np.concatenate([f, g])
    eta, omega, K = 0.7 / np.sqrt(m + n), 1.7, 40
    tau, sigma = eta / omega, eta * omega
    x = np.zeros(m * n)
    y = np.zeros(m + n)
    xs = []
    for _ in range(K):        # Algorithm 1, one PDHG step per pass
        xn = np.maximum(0.0, x - tau * (c - A.T @ y))
        y = y + sigma * (b - A @ (2.0 * xn - x))
        x = xn
        xs.append(x)
    X, p, q, res, _, Xavg = orc.solve(C, f, g, tol=0.0, max_iters=K, step_rule=orc.STEP_CONSTANT,
                                      restart_rule=orc.RESTART_NONE, eta0=eta, omega0=omega,
                                      output=1, want_average=True)
    assert res["iterations"] == K and res["status"] == 4
    np.testing.assert_allclose(vec(X), x, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(np.concatenate([p, q]), y, rtol=1e-12, atol=1e-15)
    # constant eta: the Algorithm 2 average is the arithmetic mean of the iterates
    np.testing.assert_allclose(vec(Xavg), np.mean(xs, axis=0), rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------- P-2, P-3

def test_matrix_free_products_match_kronecker_A(orc):
    rng = np.random.default_rng(3)
    m, n = 6, 9
    A = kron_A(m, n)
    X = rng.normal(size=(m, n))
    p, q = rng.normal(size=m), rng.normal(size=n)
    r, c = orc.apply_A(X)
    np.testing.assert_allclose(np.concatenate([r, c]), A @ vec(X), rtol=1e-14, atol=1e-14)
    At = orc.apply_AT(p, q)
    np.testing.assert_allclose(vec(At), A.T @ np.concatenate([p, q]), rtol=1e-14, atol=1e-14)
    # adjoint identity <X, A^T y> = <A x, y>
    lhs = float((X * At).sum())
    rhs = float(p @ r + q @ c)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


@pytest.mark.parametrize("m,n", [(7, 7), (5, 13), (1, 4)])
def test_operator_norm_is_sqrt_m_plus_n(orc, m, n):
    rng = np.random.default_rng(m + 100 * n)
    X = rng.uniform(size=(m, n))
    for _ in range(200):                   # power iteration on A^T A
        r, c = orc.apply_A(X)
        X = orc.apply_AT(r, c)
        X /= np.linalg.norm(X)
    r, c = orc.apply_A(X)
    est = np.sqrt(r @ r + c @ c)
    assert abs(est - np.sqrt(m + n)) <= 1e-9 * np.sqrt(m + n)
    ones = np.ones((m, n)) / np.sqrt(m * n)   # the maximiser named by the proposition
    r, c = orc.apply_A(ones)
    assert abs(np.sqrt(r @ r + c @ c) - np.sqrt(m + n)) <= 1e-12 * np.sqrt(m + n)


def test_step_bound_never_below_inverse_norm(orc):
    """|dy^T A dx| <= ||A|| ||dx|| ||dy|| and AM-GM give eta_bar >= 1/sqrt(m+n)."""
    inst = gen.points_sqeuclid(4, 24, 31)
    C = inst.dense_cost()
    _, _, _, res, trace = orc.solve(C, inst.f, inst.g, tol=1e-7, trace_cap=200000)
    bound = 1.0 / np.sqrt(inst.m + inst.n)
    etabars = [t["eta_bar"] for t in trace if np.isfinite(t["eta_bar"])]
    assert len(etabars) > 50
    assert min(etabars) >= bound * (1.0 - 1e-12)
    # the first step uses eta0 = 1/||A|| and is therefore accepted
    assert trace[0]["accepted"] == 1 and abs(trace[0]["eta_used"] - bound) < 1e-15


# ---------------------------------------------------------------- P-4 exact optima

@pytest.mark.parametrize("seed", range(8))
def test_objective_matches_network_simplex_tiny(orc, seed):
    rng = np.random.default_rng(1000 + seed)
    m, n = int(rng.integers(1, 9)), int(rng.integers(1, 9))
    C, f, g = random_instance(rng, m, n)
    opt, Xs = exact_lp.transport_simplex(C, f, g)
    np.testing.assert_allclose(Xs.sum(1), f, atol=1e-14)
    X, p, q, res, _ = orc.solve(C, f, g, tol=1e-9, max_iters=400000)
    assert res["status"] == 0
    assert abs(res["objective"] - opt) <= 1e-7 * max(abs(opt), 1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_network_simplex_agrees_with_highs(seed):
    """Cross-check of the two exact solvers themselves."""
    rng = np.random.default_rng(2000 + seed)
    C, f, g = random_instance(rng, 7, 5)
    opt, _ = exact_lp.transport_simplex(C, f, g)
    ref, _ = highs_opt(C, f, g)
    assert abs(opt - ref) <= 1e-12


@pytest.mark.parametrize("n", [3, 5, 7])
def test_objective_matches_permutation_brute_force(orc, n):
    rng = np.random.default_rng(50 + n)
    C = rng.uniform(size=(n, n))
    f = np.full(n, 1.0 / n)
    opt = exact_lp.assignment_brute_force(C)
    X, p, q, res, _ = orc.solve(C, f, f.copy(), tol=1e-9, max_iters=400000)
    assert res["status"] == 0
    assert abs(res["objective"] - opt) <= 1e-7 * opt


def test_objective_matches_w1_closed_form(orc):
    rng = np.random.default_rng(77)
    n, h = 40, 0.05
    f = rng.uniform(0.1, 1.0, n); f /= f.sum()
    g = rng.uniform(0.1, 1.0, n); g /= g.sum()
    pos = h * np.arange(n)
    C = np.abs(pos[:, None] - pos[None, :])
    ref = exact_lp.w1_line_closed_form(f, g, h)
    X, p, q, res, _ = orc.solve(C, f, g, tol=1e-9, max_iters=400000)
    assert res["status"] == 0
    assert abs(res["objective"] - ref) <= 1e-7 * ref


def test_objective_matches_monotone_coupling(orc):
    rng = np.random.default_rng(78)
    m, n = 120, 90
    x = rng.uniform(size=m)
    y = rng.uniform(size=n)
    f = rng.uniform(0.1, 1.0, m); f /= f.sum()
    g = rng.uniform(0.1, 1.0, n); g /= g.sum()
    C = (x[:, None] - y[None, :]) ** 2
    ref = exact_lp.monotone_coupling(x, f, y, g, lambda d: d * d)
    X, p, q, res, _ = orc.solve(C, f, g, tol=1e-9, max_iters=400000)
    assert res["status"] == 0
    assert abs(res["objective"] - ref) <= 1e-6 * ref


def test_objective_matches_highs_config1_size(orc):
    inst = gen.config_instance(1, 0)
    C = inst.dense_cost()
    ref, _ = highs_opt(C, inst.f, inst.g)
    X, p, q, res, _ = orc.solve(C, inst.f, inst.g, tol=1e-9, max_iters=400000)
    assert res["status"] == 0
    assert abs(res["objective"] - ref) <= 1e-7 * ref


def test_kkt_of_exact_lp_solution_is_zero(orc):
    """HiGHS' optimal primal and dual solutions have (near) zero relative KKT."""
    rng = np.random.default_rng(5)
    C, f, g = random_instance(rng, 6, 8)
    ref, lp = highs_opt(C, f, g)
    X = lp.x.reshape(6, 8)
    y = lp.eqlin.marginals
    parts = orc.kkt(C, f, g, X, y[:6], y[6:])
    assert parts["rel_kkt"] < 1e-9
    assert abs(parts["objective"] - ref) < 1e-12
    # a perturbed plan is detected by the primal block
    parts = orc.kkt(C, f, g, X * 1.01, y[:6], y[6:])
    assert parts["rel_primal"] > 1e-3


# ---------------------------------------------------------------- degenerate cases

def test_single_row_plan_is_forced(orc):
    rng = np.random.default_rng(9)
    n = 11
    C = rng.uniform(size=(1, n))
    g = rng.uniform(0.1, 1, n); g /= g.sum()
    X, p, q, res, _ = orc.solve(C, np.array([1.0]), g, tol=1e-10, max_iters=400000)
    assert res["status"] == 0
    np.testing.assert_allclose(X[0], g, atol=1e-9)
    X, p, q, res, _ = orc.solve(C.T.copy(), g, np.array([1.0]), tol=1e-10, max_iters=400000)
    np.testing.assert_allclose(X[:, 0], g, atol=1e-9)


def test_separable_cost_optimum(orc):
    rng = np.random.default_rng(10)
    m, n = 9, 12
    a, b = rng.uniform(size=m), rng.uniform(size=n)
    C = a[:, None] + b[None, :]
    _, f, g = random_instance(rng, m, n)
    X, p, q, res, _ = orc.solve(C, f, g, tol=1e-10, max_iters=400000)
    assert res["status"] == 0
    assert abs(res["objective"] - (a @ f + b @ g)) <= 1e-8


# ---------------------------------------------------------------- P-6 invariants

def test_dual_sums_stay_equal(orc):
    inst = gen.points_sqeuclid(2, 30, 41)
    C = inst.dense_cost()
    X, p, q, res, _ = orc.solve(C, inst.f, inst.g, tol=1e-7)
    assert abs(p.sum() - q.sum()) <= 1e-10 * (np.abs(p).sum() + np.abs(q).sum())


def test_cost_shift_and_transpose(orc):
    inst = gen.points_sqeuclid(3, 25, 33)
    C = inst.dense_cost()
    f, g = inst.f, inst.g
    _, _, _, r0, _ = orc.solve(C, f, g, tol=1e-9, max_iters=400000)
    rng = np.random.default_rng(0)
    a, b = rng.uniform(size=25), rng.uniform(size=33)
    _, _, _, r1, _ = orc.solve(C + a[:, None] + b[None, :], f, g, tol=1e-9, max_iters=400000)
    assert abs(r1["objective"] - (r0["objective"] + a @ f + b @ g)) <= 1e-7
    Xt, _, _, r2, _ = orc.solve(C.T.copy(), g, f, tol=1e-9, max_iters=400000)
    assert abs(r2["objective"] - r0["objective"]) <= 1e-7 * r0["objective"]


def test_power_of_two_scaling_is_exact(orc):
    """(C,f,g) -> s(C,f,g) scales every iterate by s (scaled-LP identity); with s = 4 the
    whole trajectory is bit-identical up to the factor, including eta_bar and omega."""
    inst = gen.points_sqeuclid(5, 20, 27)
    C = inst.dense_cost()
    X0, p0, q0, r0, t0 = orc.solve(C, inst.f, inst.g, tol=1e-7, trace_cap=100000)
    X1, p1, q1, r1, t1 = orc.solve(4.0 * C, 4.0 * inst.f, 4.0 * inst.g, tol=1e-7,
                                   trace_cap=100000)
    assert r0["iterations"] == r1["iterations"] and r0["restarts"] == r1["restarts"]
    assert np.array_equal(4.0 * X0, X1)
    assert np.array_equal(4.0 * p0, p1) and np.array_equal(4.0 * q0, q1)
    assert [t["eta_bar"] for t in t0] == [t["eta_bar"] for t in t1]
    assert r0["omega"] == r1["omega"]


# ---------------------------------------------------------------- P-7 primal weight

def test_primal_weight_is_geometric_mean_at_theta_half(orc):
    """At theta = 1/2 the update is omega' = sqrt(omega * Dy/Dx).  Restart (iii) fires at
    T=1 (k=1 >= 0.36) and T=2 (k=1 >= 0.72).  From X=0 the first step leaves X=0 (C >= 0),
    so the first restart keeps omega (Dx = 0 is guarded); the second uses the first
    restart point as its anchor."""
    inst = gen.points_sqeuclid(6, 16, 16)
    C = inst.dense_cost()
    X1, p1, q1, r1, tr1 = orc.solve(C, inst.f, inst.g, tol=1e-12, max_iters=1, output=1,
                                    trace_cap=10)
    assert r1["restarts"] == 1 and tr1[0]["restart"] == 3
    assert np.all(X1 == 0.0) and r1["omega"] == 1.0
    X2, p2, q2, r2, tr2 = orc.solve(C, inst.f, inst.g, tol=1e-12, max_iters=2, output=1,
                                    trace_cap=10)
    assert r2["restarts"] == 2 and tr2[1]["restart"] == 3
    dX = np.linalg.norm(X2 - X1)
    dY = np.sqrt(np.sum((p2 - p1) ** 2) + np.sum((q2 - q1) ** 2))
    assert dX > 0
    assert abs(r2["omega"] - np.sqrt(1.0 * dY / dX)) <= 1e-13 * r2["omega"]


# ---------------------------------------------------------------- P-9 rounding, P-5 bracket

def test_rounding_lemma_and_certified_bracket(orc):
    inst = gen.points_sqeuclid(7, 40, 35)
    C = inst.dense_cost()
    f, g = inst.f, inst.g
    X, p, q, res, _ = orc.solve(C, f, g, tol=1e-3)
    Xf = orc.round_plan(f, g, X)
    assert Xf.min() >= -1e-15 * Xf.max()   # exact arithmetic gives >= 0; FP leaves ulps
    np.testing.assert_allclose(Xf.sum(1), f, atol=1e-15)
    np.testing.assert_allclose(Xf.sum(0), g, atol=1e-15)
    viol = np.abs(f - X.sum(1)).sum() + np.abs(g - X.sum(0)).sum()
    assert np.abs(Xf - X).sum() <= 2.0 * viol * (1 + 1e-12)
    opt, _ = highs_opt(C, f, g)
    lb = orc.dual_lower_bound(C, f, g, p)
    ub = float((C * Xf).sum())
    assert lb <= opt + 1e-15 and opt <= ub + 1e-15
