"""FP64 CPU oracle for restarted PDHG on discrete optimal transport.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path (the HIP library and its
binding) never imports this package.

The arithmetic lives in ``pdhg_oracle.c`` (plain C, FP64).  This module only
marshals numpy arrays into it.  Paper: Lu & Yang, "PDOT" (arXiv 2407.19689);
Algorithm 2 (alg:rpd), the KKT error of Section 3.1, the enhancements of
Section 5, the rounding of Algorithm 3.
"""
import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

KKT_SCALED = 0      # reading R1: each block over its own scale
KKT_CUPDLP = 1      # denominators 1+||b||, 1+||C||_F, 1+|pobj|+|dobj|
STEP_ADAPTIVE = 0
STEP_CONSTANT = 1
RESTART_PDOT = 0
RESTART_BASIC = 1
RESTART_NONE = 2


class OrcParams(ct.Structure):
    _fields_ = [
        ("tol", ct.c_double),
        ("max_iters", ct.c_int64),
        ("max_passes", ct.c_int64),
        ("time_limit_s", ct.c_double),
        ("kkt_mode", ct.c_int32),
        ("step_rule", ct.c_int32),
        ("restart_rule", ct.c_int32),
        ("avg_weighting", ct.c_int32),
        ("primal_weight_update", ct.c_int32),
        ("output", ct.c_int32),
        ("beta_sufficient", ct.c_double),
        ("beta_necessary", ct.c_double),
        ("beta_artificial", ct.c_double),
        ("beta_basic", ct.c_double),
        ("theta", ct.c_double),
        ("omega0", ct.c_double),
        ("eta0", ct.c_double),
        ("eps_zero", ct.c_double),
        ("step_reduction_exp", ct.c_double),
        ("step_growth_exp", ct.c_double),
    ]


class OrcResult(ct.Structure):
    _fields_ = [
        ("status", ct.c_int32),
        ("returned_average", ct.c_int32),
        ("iterations", ct.c_int64),
        ("passes", ct.c_int64),
        ("restarts", ct.c_int64),
        ("objective", ct.c_double),
        ("dual_objective", ct.c_double),
        ("rel_primal", ct.c_double),
        ("rel_dual", ct.c_double),
        ("rel_gap", ct.c_double),
        ("rel_kkt", ct.c_double),
        ("eta", ct.c_double),
        ("omega", ct.c_double),
        ("seconds", ct.c_double),
    ]


class OrcTrace(ct.Structure):
    _fields_ = [
        ("pass_", ct.c_int64),
        ("iter", ct.c_int64),
        ("accepted", ct.c_int32),
        ("restart", ct.c_int32),
        ("cand_avg", ct.c_int32),
        ("pad", ct.c_int32),
        ("eta_used", ct.c_double),
        ("eta_bar", ct.c_double),
        ("k_cur", ct.c_double),
        ("k_avg", ct.c_double),
        ("omega", ct.c_double),
    ]


_D = ct.POINTER(ct.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ct.CDLL(_LIB_PATH)
    lib.orc_params_default.argtypes = [ct.POINTER(OrcParams)]
    lib.orc_apply_A.argtypes = [ct.c_int64, ct.c_int64, _D, _D, _D]
    lib.orc_apply_AT.argtypes = [ct.c_int64, ct.c_int64, _D, _D, _D]
    lib.orc_kkt.argtypes = [ct.c_int64, ct.c_int64, _D, _D, _D, _D, _D, _D, ct.c_int32, _D]
    lib.orc_solve.argtypes = [ct.c_int64, ct.c_int64, _D, _D, _D, ct.POINTER(OrcParams),
                              _D, _D, _D, _D, ct.POINTER(OrcResult), ct.POINTER(OrcTrace),
                              ct.c_int64, ct.c_int32]
    lib.orc_solve.restype = ct.c_int
    lib.orc_round.argtypes = [ct.c_int64, ct.c_int64, _D, _D, _D, _D]
    lib.orc_dual_lower_bound.argtypes = [ct.c_int64, ct.c_int64, _D, _D, _D, _D]
    lib.orc_dual_lower_bound.restype = ct.c_double
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params(**kw) -> OrcParams:
    """Paper defaults (Section 5: beta 0.1/0.9/0.36, theta 0.5, omega0 1;
    Section 5.1: tol 1e-4), overridden by keyword."""
    p = OrcParams()
    _load().orc_params_default(ct.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def apply_A(X):
    """A vec(X) = [X 1_n ; X^T 1_m] (Section 3.1)."""
    X = _f64(X)
    m, n = X.shape
    r = np.empty(m)
    c = np.empty(n)
    _load().orc_apply_A(m, n, _p(X), _p(r), _p(c))
    return r, c


def apply_AT(p, q):
    """A^T [p;q] = p 1_n^T + 1_m q^T (Section 3.1)."""
    p = _f64(p)
    q = _f64(q)
    out = np.empty((p.size, q.size))
    _load().orc_apply_AT(p.size, q.size, _p(p), _p(q), _p(out))
    return out


def kkt(C, f, g, X, p, q, kkt_mode=KKT_SCALED):
    """Relative KKT parts of any triple: dict with rel_primal, rel_dual, rel_gap,
    rel_kkt, objective, dual_objective, abs_primal, abs_dual."""
    C, f, g, X, p, q = map(_f64, (C, f, g, X, p, q))
    m, n = C.shape
    out = np.zeros(8)
    _load().orc_kkt(m, n, _p(C), _p(f), _p(g), _p(X), _p(p), _p(q), kkt_mode, _p(out))
    keys = ("rel_primal", "rel_dual", "rel_gap", "rel_kkt", "objective", "dual_objective",
            "abs_primal", "abs_dual")
    return dict(zip(keys, out.tolist()))


def solve(C, f, g, prm=None, nthreads=0, trace_cap=0, want_average=False, **kw):
    """Run the oracle. Returns (X, p, q, result_dict, trace_list[, Xavg])."""
    C, f, g = _f64(C), _f64(f), _f64(g)
    m, n = C.shape
    if prm is None:
        prm = params(**kw)
    X = np.zeros((m, n))
    p = np.zeros(m)
    q = np.zeros(n)
    Xa = np.zeros((m, n)) if want_average else None
    res = OrcResult()
    tr = (OrcTrace * trace_cap)() if trace_cap > 0 else None
    nt = _load().orc_solve(m, n, _p(C), _p(f), _p(g), ct.byref(prm), _p(X), _p(p), _p(q),
                           _p(Xa) if Xa is not None else None, ct.byref(res),
                           tr, trace_cap, nthreads)
    rd = {k: getattr(res, k) for k, _ in OrcResult._fields_}
    trace = []
    for i in range(nt):
        t = tr[i]
        trace.append({k.rstrip("_"): getattr(t, k) for k, _ in OrcTrace._fields_})
    if want_average:
        return X, p, q, rd, trace, Xa
    return X, p, q, rd, trace


def round_plan(f, g, X):
    """Algorithm 3: exactly feasible plan near X."""
    f, g, X = _f64(f), _f64(g), _f64(X)
    m, n = X.shape
    out = np.empty((m, n))
    _load().orc_round(m, n, _p(f), _p(g), _p(X), _p(out))
    return out


def dual_lower_bound(C, f, g, p):
    """f^T p + g^T q with q the c-transform of p: a certified lower bound on OPT."""
    C, f, g, p = map(_f64, (C, f, g, p))
    m, n = C.shape
    return _load().orc_dual_lower_bound(m, n, _p(C), _p(f), _p(g), _p(p))
