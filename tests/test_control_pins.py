"""Pins of the oracle's Section 5 control: step size, restarts, primal weight, termination.

The oracle (oracle/pdhg_oracle.c) runs Algorithm 2 in matrix form.  The reference below is
written separately from the paper's text in the vector form of Algorithm 1 (Section 2): the
LP  min c^T x  s.t.  A x = b, x >= 0  with the explicit Kronecker matrix
A = [1_n^T kron I_m ; I_n kron 1_m^T], c = vec(C), b = [f; g] (Section 3.1, eq.
ot-lp-data), and the KKT error from the LP form (primal residual ||Ax - b||, dual residual
||[A^T y - c]^+||, gap c^T x - b^T y).  Its control follows Section 5:

  * step size: tau = eta/omega, sigma = eta*omega; a trial is accepted when
        eta <= (omega ||dx||^2 + ||dy||^2 / omega) / (2 |dy^T A dx|)
    (the squared weighted norm of the cited PDLP rule; +inf when the denominator is 0),
    and after every trial eta becomes min((1 - (T+1)^-0.3) eta_bar, (1 + (T+1)^-0.6) eta)
    with T the accepted iterations so far (PDLP's published constants, typed here
    independently of the oracle's parameters); a rejected trial is retried from the same
    point;
  * average weighted by the step used (uniform when eta is constant, Algorithm 2), kept
    here as a weighted sum and a weight total rather than the running update;
  * restart candidate: the current point when its KKT is strictly lower, else the average;
  * restart when (i) K_c <= beta_sufficient K_start, or (ii) K_c <= beta_necessary K_start
    and K_c > K_c of the previous iteration, or (iii) k >= beta_artificial T; move to the
    candidate, primal weight exp(theta log(Dy/Dx) + (1-theta) log omega) when both
    distances from the previous restart point exceed eps_zero;
  * Algorithm 2's own rule (restart_rule 1): restart to the average when
    KKT(average) <= beta KKT(restart point) (eq. restart-condition);
  * stop when the candidate's relative KKT is at most tol (Section 5.1).

The readings where the paper is silent (relative KKT scales, start point, tie rule,
K_prev after a restart, total_iteration = accepted iterations) are the ones the oracle
documents; everything else here is the paper's statement, so a dropped term, a swapped
exponent or beta, or a wrong counter in the oracle changes the trace it is compared with.
"""
import math

import numpy as np
import pytest

from tests.trace_walk import walk_traces
from workloads import generators as gen

# PDLP's step-size constants (Applegate et al. 2021), cited by Section 5.
PDLP_REDUCTION = 0.3
PDLP_GROWTH = 0.6


def kron_A(m, n):
    return np.vstack([np.kron(np.ones((1, n)), np.eye(m)), np.kron(np.eye(n), np.ones((1, m)))])


def vec(X):
    return X.reshape(-1, order="F")


def unvec(x, m, n):
    return x.reshape((n, m)).T


class ExplicitPDHG:
    """Restarted PDHG on the explicit LP (Algorithm 1 + Section 5)."""

    def __init__(self, C, f, g, kkt_mode=0, step_rule=0, restart_rule=0, avg_uniform=False,
                 beta_sufficient=0.1, beta_necessary=0.9, beta_artificial=0.36,
                 beta_basic=0.2, theta=0.5, omega0=1.0, eta0=None, eps_zero=1e-10,
                 reduction=PDLP_REDUCTION, growth=PDLP_GROWTH, primal_weight_update=True):
        self.m, self.n = C.shape
        self.A = kron_A(self.m, self.n)
        self.c = vec(C)
        self.b = np.concatenate([f, g])
        self.kkt_mode = kkt_mode
        self.step_rule = step_rule
        self.restart_rule = restart_rule
        self.avg_uniform = avg_uniform
        self.bs, self.bn, self.ba, self.bb = beta_sufficient, beta_necessary, beta_artificial, beta_basic
        self.theta, self.eps = theta, eps_zero
        self.red, self.grow = reduction, growth
        self.pwu = primal_weight_update
        self.omega = omega0
        self.eta = eta0 if eta0 is not None else 1.0 / math.sqrt(self.m + self.n)

    def kkt(self, x, y):
        """Relative KKT from the LP form: each block over its scale (kkt_mode 0) or over
        1 + scale (kkt_mode 1), combined as a 2-norm."""
        A, b, c = self.A, self.b, self.c
        prim = np.linalg.norm(A @ x - b)
        dual = np.linalg.norm(np.maximum(A.T @ y - c, 0.0))
        pobj, dobj = float(c @ x), float(b @ y)
        gap = abs(pobj - dobj)
        nb, nc = np.linalg.norm(b), np.linalg.norm(c)
        if self.kkt_mode == 1:
            parts = (prim / (1 + nb), dual / (1 + nc), gap / (1 + abs(pobj) + abs(dobj)))
        else:
            den = abs(pobj) + abs(dobj)
            parts = (prim / nb if nb > 0 else prim, dual / nc if nc > 0 else dual,
                     gap / den if den > 0 else 0.0)
        return math.sqrt(sum(v * v for v in parts))

    def run(self, tol, max_iters):
        A, b, c = self.A, self.b, self.c
        x = np.zeros(A.shape[1])
        y = np.zeros(A.shape[0])
        trace = []
        T = k = passes = 0
        wsum, xs, ys = 0.0, np.zeros_like(x), np.zeros_like(y)
        x_anchor, y_anchor = x.copy(), y.copy()
        K_start = K_prev = self.kkt(x, y)
        cand = (x, y)
        if K_start <= tol:
            return x, y, trace, dict(T=0, restarts=0, converged=True, omega=self.omega)
        restarts = 0
        converged = False
        while T < max_iters:
            while True:                     # trials from the same point until accepted
                passes += 1
                tau, sigma = self.eta / self.omega, self.eta * self.omega
                xn = np.maximum(0.0, x - tau * (c - A.T @ y))
                yn = y + sigma * (b - A @ (2.0 * xn - x))
                used = self.eta
                if self.step_rule == 1:
                    eta_bar, ok = math.inf, True
                else:
                    dx, dy = xn - x, yn - y
                    num = self.omega * float(dx @ dx) + float(dy @ dy) / self.omega
                    den = 2.0 * abs(float(dy @ (A @ dx)))
                    eta_bar = num / den if den > 0 else math.inf
                    ok = used <= eta_bar
                    # an infinite bound limits nothing (at T = 0 its factor is 0)
                    shrink = (math.inf if math.isinf(eta_bar)
                              else (1.0 - (T + 1) ** (-self.red)) * eta_bar)
                    self.eta = min(shrink, (1.0 + (T + 1) ** (-self.grow)) * used)
                if ok:
                    break
                trace.append(dict(pass_=passes, iter=T, accepted=0, restart=0, cand_avg=0,
                                  eta_used=used, eta_bar=eta_bar, omega=self.omega))
            x, y = xn, yn
            T += 1
            k += 1
            w = 1.0 if self.avg_uniform else used
            wsum += w
            xs = xs + w * x
            ys = ys + w * y
            if k == 1:                      # the average of one iterate is that iterate,
                xbar, ybar = x, y           # so its KKT ties with the current one exactly
            else:
                xbar, ybar = xs / wsum, ys / wsum
            k_cur, k_avg = self.kkt(x, y), self.kkt(xbar, ybar)
            cand_avg = not (k_cur < k_avg)
            K_c = k_avg if cand_avg else k_cur
            kind = 0
            if K_c <= tol:
                converged = True
            elif self.restart_rule == 0:
                if K_c <= self.bs * K_start:
                    kind = 1
                elif K_c <= self.bn * K_start and K_c > K_prev:
                    kind = 2
                elif k >= self.ba * T:
                    kind = 3
            elif self.restart_rule == 1:
                if k_avg <= self.bb * K_start:
                    kind, cand_avg, K_c = 1, True, k_avg
            trace.append(dict(pass_=passes, iter=T, accepted=1, restart=kind,
                              cand_avg=int(cand_avg), eta_used=used, eta_bar=eta_bar,
                              k_cur=k_cur, k_avg=k_avg, omega=self.omega))
            cand = (xbar, ybar) if cand_avg else (x, y)
            if converged:
                break
            if kind:
                x, y = cand[0].copy(), cand[1].copy()
                Dx = np.linalg.norm(x - x_anchor)
                Dy = np.linalg.norm(y - y_anchor)
                if self.pwu and Dx > self.eps and Dy > self.eps:
                    self.omega = math.exp(self.theta * math.log(Dy / Dx)
                                          + (1.0 - self.theta) * math.log(self.omega))
                x_anchor, y_anchor = x.copy(), y.copy()
                wsum, xs, ys = 0.0, np.zeros_like(x), np.zeros_like(y)
                k = 0
                restarts += 1
                K_start = K_prev = K_c
                cand = (x, y)
            else:
                K_prev = K_c
        return cand[0], cand[1], trace, dict(T=T, restarts=restarts, converged=converged,
                                             omega=self.omega, passes=passes)


def tiny(seed, m, n):
    inst = gen.points_sqeuclid(seed, m, n)
    return inst.dense_cost(), inst.f, inst.g


def oracle_kwargs(ref):
    return dict(kkt_mode=ref.kkt_mode, step_rule=ref.step_rule, restart_rule=ref.restart_rule,
                avg_weighting=1 if ref.avg_uniform else 0, beta_sufficient=ref.bs,
                beta_necessary=ref.bn, beta_artificial=ref.ba, beta_basic=ref.bb,
                theta=ref.theta, omega0=ref.omega, eps_zero=ref.eps,
                primal_weight_update=1 if ref.pwu else 0)


def compare(orc, C, f, g, iters=300, tol=1e-12, drift_cap=1e-6, **kw):
    """Run both on the same instance and walk the two traces together (walk_traces): over
    the prefix in which their scalars agree to drift_cap every decision must be identical.
    Returns the compared reference entries and the final states."""
    ref = ExplicitPDHG(C, f, g, **kw)
    okw = oracle_kwargs(ref)
    okw["eta0"] = ref.eta
    xr, yr, tr_ref, info = ref.run(tol, iters)
    X, p, q, res, tr = orc.solve(C, f, g, tol=tol, max_iters=iters, trace_cap=100000,
                                 nthreads=1, step_reduction_exp=0.3, step_growth_exp=0.6,
                                 **okw)
    compared = walk_traces(tr, tr_ref, drift_cap)
    if len(compared) == len(tr_ref):
        assert len(tr) == len(tr_ref)
        assert res["iterations"] == info["T"] and res["restarts"] == info["restarts"]
    return compared, (X, p, q, xr, yr, info)


def kinds(trace):
    return {t["restart"] for t in trace if t["accepted"]} - {0}


# ------------------------------------------------------------ the full control sequence

# Tiny instances on which, within the compared prefix of 300 iterations at the paper's
# constants, all three restart conditions fire and the step rule rejects a trial.
TRACE_CASES = [(8, 8, 5), (30, 3, 4), (49, 3, 5)]


@pytest.mark.parametrize("seed,m,n", TRACE_CASES)
def test_adaptive_control_trace_matches_explicit_lp(orc, seed, m, n):
    """Section 5 defaults: accept/reject passes, restart iterations and conditions,
    candidate side, eta, eta_bar, both KKT values and omega agree step for step."""
    C, f, g = tiny(seed, m, n)
    tr, _ = compare(orc, C, f, g)
    assert tr[-1]["iter"] >= 140, "the compared prefix is too short"
    assert kinds(tr) == {1, 2, 3}, "a restart condition never fired"
    assert any(t["accepted"] == 0 for t in tr), "no rejected trial: the retry path is untested"


@pytest.mark.parametrize("seed,m,n", [(5, 6, 6), (6, 5, 8)])
def test_kkt_mode_1_trace_matches_explicit_lp(orc, seed, m, n):
    """The 1 + scale denominators (kkt_mode 1) through the control sequence."""
    C, f, g = tiny(seed, m, n)
    tr, _ = compare(orc, C, f, g, kkt_mode=1)
    assert tr[-1]["iter"] >= 100 and kinds(tr)


@pytest.mark.parametrize("seed,m,n", [(7, 6, 5), (8, 9, 4)])
def test_algorithm2_basic_restart_trace_matches_explicit_lp(orc, seed, m, n):
    """Algorithm 2 as printed: restart to the average once its KKT has decayed by beta
    (eq. restart-condition), with the adaptive step, and with a constant step, uniform
    weights and a fixed primal weight, where the whole run and its final iterates agree to
    rounding."""
    C, f, g = tiny(seed, m, n)
    tr, _ = compare(orc, C, f, g, restart_rule=1, beta_basic=0.5)
    restarts = [t for t in tr if t["accepted"] and t["restart"]]
    assert len(restarts) >= 2 and all(t["cand_avg"] == 1 for t in restarts)
    eta = 1.0 / (2.0 * math.sqrt(m + n))
    tr, (X, p, q, xr, yr, info) = compare(orc, C, f, g, restart_rule=1, beta_basic=0.5,
                                          step_rule=1, avg_uniform=True, eta0=eta,
                                          primal_weight_update=False, drift_cap=1e-9)
    assert len(tr) == 300 and info["restarts"] >= 1
    assert np.abs(vec(X) - xr).max() <= 1e-12 * np.abs(xr).max()
    assert np.abs(np.concatenate([p, q]) - yr).max() <= 1e-12 * np.abs(yr).max()


@pytest.mark.parametrize("only", [1, 2])
def test_restart_conditions_i_and_ii_each_alone(orc, only):
    """With beta_artificial out of reach, and the other decay condition switched off, each
    of (i) and (ii) fires on its own and nothing else restarts."""
    C, f, g = tiny(8, 8, 5)
    kw = dict(beta_artificial=1e9)
    if only == 1:
        kw["beta_necessary"] = 0.0
    else:
        kw["beta_sufficient"] = 0.0
    tr, _ = compare(orc, C, f, g, iters=400, **kw)
    assert kinds(tr) == {only}
    _, _, _, _, full = orc.solve(C, f, g, tol=1e-12, max_iters=400, trace_cap=100000,
                                 nthreads=1, **{k: v for k, v in kw.items()})
    assert kinds(full) == {only}


def test_no_restart_when_every_condition_is_off(orc):
    C, f, g = tiny(30, 3, 4)
    tr, _ = compare(orc, C, f, g, beta_sufficient=0.0, beta_necessary=0.0,
                    beta_artificial=1e9)
    assert tr[-1]["iter"] >= 100 and not kinds(tr)
    _, _, _, res, _ = orc.solve(C, f, g, tol=1e-12, max_iters=300, nthreads=1,
                                beta_sufficient=0.0, beta_necessary=0.0, beta_artificial=1e9)
    assert res["restarts"] == 0


def test_restart_every_iteration_with_zero_artificial_beta(orc):
    """(iii) with beta_artificial = 0 holds at every k >= 1 (or (i)/(ii) fire first)."""
    C, f, g = tiny(49, 3, 5)
    tr, _ = compare(orc, C, f, g, iters=120, beta_artificial=0.0)
    assert tr[-1]["iter"] >= 60
    assert all(t["restart"] for t in tr if t["accepted"])
    _, _, _, res, _ = orc.solve(C, f, g, tol=1e-12, max_iters=120, nthreads=1,
                                beta_artificial=0.0)
    assert res["restarts"] == 120


def test_swapped_step_exponents_change_the_trace(orc):
    """The oracle run with the two PDLP exponents exchanged departs from the explicit
    reference run with the published ones (0.3 for the reduction, 0.6 for the growth)."""
    C, f, g = tiny(8, 8, 5)
    ref = ExplicitPDHG(C, f, g)
    _, _, tr_ref, _ = ref.run(1e-12, 300)
    _, _, _, _, tr = orc.solve(C, f, g, tol=1e-12, max_iters=300, trace_cap=100000,
                               nthreads=1, step_reduction_exp=0.6, step_growth_exp=0.3)
    etas = [t["eta_used"] for t in tr]
    etas_ref = [t["eta_used"] for t in tr_ref]
    n = min(len(etas), len(etas_ref))
    assert len(etas) != len(etas_ref) or max(abs(a - b) / b for a, b in zip(etas[:n], etas_ref[:n])) > 1e-3


def test_step_update_by_hand(orc):
    """The first trials by hand on a 1 x 2 problem, where everything has a closed form.

    C = [0, 1], f = [1], g = [1/2, 1/2], omega = 1, eta0 = 1/sqrt(3).  From x = 0, y = 0:
    x+ = max(0, -tau c) = 0 (C >= 0), so dx = 0 and eta_bar = +inf: accepted, and
    eta1 = min(+inf, (1 + 1^-0.6) eta0) = 2 eta0.  y+ = sigma b, so (p, q) = eta0 (1, .5, .5).
    Second trial from (0, y1) with eta = 2 eta0: x+ = max(0, tau (A^T y1 - c)),
    A^T y1 = (p + q_1, p + q_2) = 1.5 eta0 (1, 1)."""
    C = np.array([[0.0, 1.0]])
    f = np.array([1.0])
    g = np.array([0.5, 0.5])
    e0 = 1.0 / math.sqrt(3.0)
    _, _, _, _, tr = orc.solve(C, f, g, tol=1e-14, max_iters=2, trace_cap=16, nthreads=1,
                               restart_rule=2, output=1)
    assert tr[0]["accepted"] == 1 and math.isinf(tr[0]["eta_bar"]) and tr[0]["eta_used"] == e0
    e1 = 2.0 * e0
    # second trial by hand
    y1 = e0 * np.array([1.0, 0.5, 0.5])
    x1 = np.maximum(0.0, e1 * (np.array([y1[0] + y1[1], y1[0] + y1[2]]) - C[0]))
    r, cs = x1.sum(), x1                                    # A x1 = (row sum, column sums)
    y2 = y1 + e1 * (np.array([1.0, 0.5, 0.5]) - np.array([2 * r, 2 * cs[0], 2 * cs[1]]))
    dy = y2 - y1
    num = float(x1 @ x1) + float(dy @ dy)
    den = 2.0 * abs(dy[0] * r + dy[1] * cs[0] + dy[2] * cs[1])
    eta_bar = num / den
    second = tr[1]
    assert abs(second["eta_used"] - e1) <= 1e-15 * e1
    assert abs(second["eta_bar"] - eta_bar) <= 1e-13 * eta_bar
    accepted = e1 <= eta_bar
    assert second["accepted"] == int(accepted)
    nxt = min((1.0 - 2.0 ** -0.3) * eta_bar, (1.0 + 2.0 ** -0.6) * e1)
    if len(tr) > 2:
        assert abs(tr[2]["eta_used"] - nxt) <= 1e-13 * nxt


def test_termination_returns_the_candidate_that_met_tol(orc):
    """The oracle stops at the first iteration whose candidate KKT is at most tol, as the
    reference does, and returns that candidate."""
    C, f, g = tiny(9, 5, 9)
    ref = ExplicitPDHG(C, f, g)
    xr, yr, tr_ref, info = ref.run(1e-4, 100000)
    assert info["converged"]
    X, p, q, res, tr = orc.solve(C, f, g, tol=1e-4, trace_cap=200000, nthreads=1)
    assert res["status"] == 0 and res["iterations"] == info["T"]
    assert res["returned_average"] == tr_ref[-1]["cand_avg"]
    # the iterates separate slowly under the adaptive step (see compare)
    np.testing.assert_allclose(vec(X), xr, rtol=0, atol=1e-6 * np.abs(xr).max())
    np.testing.assert_allclose(np.concatenate([p, q]), yr, rtol=0, atol=1e-6 * np.abs(yr).max())
