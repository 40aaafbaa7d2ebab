"""MI355X (gfx950) restarted PDHG for discrete optimal transport.

Thin Python binding of the C ABI in ``include/pdot.h``; the names match the C entry
points.  The binding only marshals arguments: buffers come from PyTorch (device memory
and streams) or numpy (host memory), and every step of the solver runs in the HIP
library ``libpdot.so``.  Importing works without the library; the first call raises if
it has not been built.

Method: Lu & Yang, "PDOT" (arXiv 2407.19689), Algorithm 2 with the Section 5
enhancements and the Section 5.1 termination rule.
"""
import ctypes as ct

import numpy as np

from . import _abi
from ._abi import (  # noqa: F401
    OT_OK, OT_ERR_INVALID, OT_ERR_OOM, OT_ERR_DEVICE, OT_NOT_CONVERGED, OT_ERR_NUMERIC,
    OT_ERR_BUSY, OT_PREC_FP64, OT_PREC_FP32, OT_COST_DENSE, OT_COST_POINTS_SQEUCLID,
    OT_COST_POINTS_EUCLID, OT_COST_GRID_SQEUCLID, OT_COST_GRID_L1, OT_COST_GRID_L2,
    OT_COST_GRID_LINF, OT_NOALLOC_MAX_BYTES, OtCost, OtParams, OtProblem, OtResult, OtTraceRec,
    OtServerCfg, OtCompletion, OtServerStats, OtBracket, STATUS_NAMES,
)

__all__ = ["ot_params_default", "ot_workspace_size", "ot_solve", "ot_solve_noalloc",
           "ot_solve_batch", "ot_round",
           "ot_last_error", "ot_version", "ot_server_create", "ot_server_submit",
           "ot_server_poll", "ot_server_drain", "ot_server_get_stats", "ot_server_destroy",
           "params", "problem", "solve_instance", "problem_from_instance", "Server"]


def _ptr(a):
    """Address of a torch tensor, numpy array or None (argument marshalling only)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data
    raise TypeError(f"unsupported buffer type {type(a)}")


def _check_f64(a, name):
    if a is None:
        return
    dt = getattr(a, "dtype", None)
    if str(dt) not in ("float64", "torch.float64"):
        raise TypeError(f"{name} must be float64, got {dt}")


def ot_params_default() -> OtParams:
    p = OtParams()
    _abi.load().ot_params_default(ct.byref(p))
    return p


def params(**kw) -> OtParams:
    """ot_params_default() with keyword overrides (field names of ot_params)."""
    p = ot_params_default()
    for k, v in kw.items():
        if not any(k == f for f, _ in OtParams._fields_):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Problem:
    """An OtProblem plus references to the buffers it points into."""

    def __init__(self, raw: OtProblem, keep, trace_buf=None):
        self.raw = raw
        self.keep = keep
        self.trace_buf = trace_buf

    def trace(self, count):
        """The first `count` control records (ot_result.trace_len) as dicts."""
        out = []
        for i in range(min(count, len(self.trace_buf) if self.trace_buf is not None else 0)):
            r = self.trace_buf[i]
            out.append({k.rstrip("_"): getattr(r, k) for k, _ in OtTraceRec._fields_})
        return out


def problem(kind, m, n, f, g, C=None, ldc=None, x=None, y=None, side=0, scale=1.0,
            store=0, tol=0.0, X_out=None, u_out=None, v_out=None, tile_vec=0,
            tile_rows=0, trace_cap=0) -> Problem:
    """Build an ot_problem from torch tensors or numpy arrays (host or device).
    trace_cap > 0 gives the problem a host buffer for that many control records."""
    for a, nm in ((f, "f"), (g, "g"), (C, "C"), (x, "x"), (y, "y"), (u_out, "u_out"),
                  (v_out, "v_out")):
        _check_f64(a, nm)
    c = OtCost()
    c.kind = kind
    c.store = store
    c.scale = scale
    c.side = side
    if C is not None:
        c.C = _ptr(C)
        c.ldc = ldc if ldc is not None else n
    if x is not None:
        c.x = _ptr(x)
        c.y = _ptr(y)
        c.dim = int(x.shape[1]) if len(x.shape) == 2 else 1
    pr = OtProblem()
    pr.cost = c
    pr.m = m
    pr.n = n
    pr.f = _ptr(f)
    pr.g = _ptr(g)
    pr.tol = tol
    pr.X_out = _ptr(X_out)
    pr.u_out = _ptr(u_out)
    pr.v_out = _ptr(v_out)
    pr.tile_vec = tile_vec
    pr.tile_rows = tile_rows
    tbuf = None
    if trace_cap > 0:
        tbuf = (OtTraceRec * trace_cap)()
        pr.trace = ct.addressof(tbuf)
        pr.trace_cap = trace_cap
    return Problem(pr, [f, g, C, x, y, X_out, u_out, v_out], tbuf)


def ot_workspace_size(prob: Problem, prm: OtParams) -> int:
    return int(_abi.load().ot_workspace_size(ct.byref(prob.raw), ct.byref(prm)))


def ot_solve(prob: Problem, prm: OtParams, workspace=None, stream=None):
    """Returns (status, OtResult)."""
    res = OtResult()
    ws = _ptr(workspace)
    nbytes = 0
    if workspace is not None:
        nbytes = workspace.numel() * workspace.element_size() if hasattr(workspace, "numel") \
            else workspace.nbytes
    st = _abi.load().ot_solve(ct.byref(prob.raw), ct.byref(prm), ct.byref(res), ws, nbytes,
                              stream)
    return int(st), res


def ot_solve_noalloc(prob: Problem, prm: OtParams, stream=None):
    """ot_solve on the library's static device array (no allocation).  Returns
    (status, OtResult)."""
    res = OtResult()
    st = _abi.load().ot_solve_noalloc(ct.byref(prob.raw), ct.byref(prm), ct.byref(res), stream)
    return int(st), res


def ot_solve_batch(probs, prm: OtParams, stream=None):
    """Returns (status, [OtResult])."""
    arr = (OtProblem * len(probs))(*[p.raw for p in probs])
    res = (OtResult * len(probs))()
    st = _abi.load().ot_solve_batch(arr, len(probs), ct.byref(prm), res, stream)
    return int(st), list(res)


def ot_round(prob: Problem, precision, X, u, X_feas=None, stream=None):
    """Algorithm 3 on the plan X and the certified bracket from the duals u.
    Returns (status, dict with upper, lower, l1_change, marginal_l1, feas_violation)."""
    out = OtBracket()
    _check_f64(u, "u")
    _check_f64(X_feas, "X_feas")
    st = _abi.load().ot_round(ct.byref(prob.raw), precision, _ptr(X), _ptr(u), _ptr(X_feas),
                              ct.byref(out), stream)
    return int(st), out.as_dict()


def ot_server_create(hbm_budget_bytes, max_active=64, max_queue=0, block_ms=0.0, prm=None):
    """Returns (status, handle)."""
    cfg = OtServerCfg()
    cfg.hbm_budget_bytes = int(hbm_budget_bytes)
    cfg.max_active = max_active
    cfg.max_queue = max_queue
    cfg.block_ms = block_ms
    cfg.params = prm if prm is not None else ot_params_default()
    h = ct.c_void_p()
    st = _abi.load().ot_server_create(ct.byref(cfg), ct.byref(h))
    return int(st), h


def ot_server_submit(handle, prob: Problem):
    """Returns (status, ticket)."""
    t = ct.c_uint64()
    st = _abi.load().ot_server_submit(handle, ct.byref(prob.raw), ct.byref(t))
    return int(st), int(t.value)


def ot_server_poll(handle, max_n=256):
    """Returns (status, [OtCompletion])."""
    buf = (OtCompletion * max_n)()
    n = ct.c_int32()
    st = _abi.load().ot_server_poll(handle, buf, max_n, ct.byref(n))
    return int(st), [buf[i] for i in range(n.value)]


def ot_server_drain(handle, timeout_s=0.0):
    return int(_abi.load().ot_server_drain(handle, timeout_s))


def ot_server_get_stats(handle):
    o = OtServerStats()
    st = _abi.load().ot_server_get_stats(handle, ct.byref(o))
    return int(st), {k: getattr(o, k) for k, _ in OtServerStats._fields_}


def ot_server_destroy(handle):
    return int(_abi.load().ot_server_destroy(handle))


class Server:
    """Owner of an ot_server handle that keeps every submitted problem's buffers alive until
    its completion has been polled."""

    def __init__(self, hbm_budget_bytes, max_active=64, max_queue=0, block_ms=0.0, prm=None, **kw):
        if prm is None:
            prm = params(**kw)
        st, self.handle = ot_server_create(hbm_budget_bytes, max_active, max_queue, block_ms, prm)
        if st != OT_OK:
            raise RuntimeError(f"ot_server_create: {STATUS_NAMES.get(st)} {ot_last_error()}")
        self.live = {}

    def submit(self, prob: Problem):
        st, t = ot_server_submit(self.handle, prob)
        if st == OT_OK:
            self.live[t] = prob
        return st, t

    def poll(self, max_n=256):
        st, out = ot_server_poll(self.handle, max_n)
        res = []
        for c in out:
            d = c.result.as_dict()
            d.update(ticket=c.ticket, t_submit=c.t_submit, t_admit=c.t_admit, t_done=c.t_done)
            res.append(d)
            self.live.pop(c.ticket, None)
        return res

    def drain(self, timeout_s=0.0):
        return ot_server_drain(self.handle, timeout_s)

    def stats(self):
        return ot_server_get_stats(self.handle)[1]

    def close(self):
        if self.handle:
            ot_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def ot_last_error() -> str:
    return _abi.load().ot_last_error().decode()


def ot_version() -> str:
    return _abi.load().ot_version().decode()


# ------------------------------------------------------------------ convenience

_KINDS = {
    "points_sqeuclid": OT_COST_POINTS_SQEUCLID,
    "points_euclid": OT_COST_POINTS_EUCLID,
    "grid_sqeuclid": OT_COST_GRID_SQEUCLID,
    "grid_l1": OT_COST_GRID_L1,
    "grid_l2": OT_COST_GRID_L2,
    "grid_linf": OT_COST_GRID_LINF,
}


def problem_from_instance(inst, device="cuda", precision=OT_PREC_FP32, store=0, dense=False,
                          tol=0.0, want_plan=True, tile_vec=0, tile_rows=0, trace_cap=0):
    """Place an instance (attributes m, n, f, g, kind, x, y, side, scale, dense_cost())
    in device memory with torch and allocate the outputs.  Returns (Problem, outputs)."""
    import torch
    dev = torch.device(device)
    f = torch.as_tensor(np.ascontiguousarray(inst.f, dtype=np.float64), device=dev)
    g = torch.as_tensor(np.ascontiguousarray(inst.g, dtype=np.float64), device=dev)
    xdt = torch.float32 if precision == OT_PREC_FP32 else torch.float64
    X = torch.empty((inst.m, inst.n), dtype=xdt, device=dev) if want_plan else None
    u = torch.empty(inst.m, dtype=torch.float64, device=dev)
    v = torch.empty(inst.n, dtype=torch.float64, device=dev)
    out = {"X": X, "u": u, "v": v}
    if dense or inst.kind not in _KINDS:
        C = torch.as_tensor(np.ascontiguousarray(inst.dense_cost(), dtype=np.float64), device=dev)
        pr = problem(OT_COST_DENSE, inst.m, inst.n, f, g, C=C, tol=tol, X_out=X, u_out=u, v_out=v,
                     tile_vec=tile_vec, tile_rows=tile_rows, trace_cap=trace_cap)
        return pr, out
    kind = _KINDS[inst.kind]
    if kind in (OT_COST_GRID_SQEUCLID, OT_COST_GRID_L1, OT_COST_GRID_L2, OT_COST_GRID_LINF):
        pr = problem(kind, inst.m, inst.n, f, g, side=inst.side, scale=inst.scale, store=store,
                     tol=tol, X_out=X, u_out=u, v_out=v, tile_vec=tile_vec, tile_rows=tile_rows,
                     trace_cap=trace_cap)
    else:
        x = torch.as_tensor(np.ascontiguousarray(inst.x, dtype=np.float64), device=dev)
        y = torch.as_tensor(np.ascontiguousarray(inst.y, dtype=np.float64), device=dev)
        pr = problem(kind, inst.m, inst.n, f, g, x=x, y=y, store=store, tol=tol, X_out=X,
                     u_out=u, v_out=v, tile_vec=tile_vec, tile_rows=tile_rows,
                     trace_cap=trace_cap)
    return pr, out


def solve_instance(inst, prm: OtParams = None, device="cuda", store=0, dense=False, tol=0.0,
                   stream=None, trace_cap=0, **kw):
    """ot_solve on one instance; returns (status, result dict, outputs dict of tensors).
    With trace_cap > 0 the outputs also hold the control records under "trace"."""
    if prm is None:
        prm = params(**kw)
    pr, out = problem_from_instance(inst, device=device, precision=prm.precision, store=store,
                                    dense=dense, tol=tol, trace_cap=trace_cap)
    st, res = ot_solve(pr, prm, stream=stream)
    if trace_cap > 0:
        out["trace"] = pr.trace(res.trace_len)
    return st, res.as_dict(), out
