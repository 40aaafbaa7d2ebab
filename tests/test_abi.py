"""C-ABI checks that need no GPU: the library loads, exports every entry point that
include/pdot.h declares, the ctypes mirror has the C layout, defaults are the paper's
constants, and invalid problems are rejected before any device call."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2407_19689_amd as P
from paper_2407_19689_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdot.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ot_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    names = declared_functions()
    assert "ot_solve" in names and "ot_solve_batch" in names
    for nm in names:
        assert hasattr(lib, nm), nm
    # and the binding wraps each of them
    for nm in names:
        assert nm in _abi.SIGNATURES, nm


def test_ctypes_structs_match_c_layout(tmp_path):
    src = tmp_path / "layout.c"
    cls = {"ot_cost": P.OtCost, "ot_problem": P.OtProblem, "ot_params": P.OtParams,
           "ot_result": P.OtResult, "ot_server_cfg": P.OtServerCfg,
           "ot_completion": P.OtCompletion, "ot_server_stats": P.OtServerStats,
           "ot_bracket": P.OtBracket, "ot_trace_rec": P.OtTraceRec}
    fields = {st: [f for f, _ in c._fields_] for st, c in cls.items()}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void){']
    for st, fl in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fl:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f.rstrip("_")}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    for st, c in cls.items():
        assert int(got[st]) == ct.sizeof(c), st
        for f in fields[st]:
            assert int(got[f"{st}.{f}"]) == getattr(c, f).offset, (st, f)


def test_defaults_are_the_paper_constants():
    p = P.ot_params_default()
    # Section 5: adaptive restart parameters and primal weight
    assert (p.beta_sufficient, p.beta_necessary, p.beta_artificial) == (0.1, 0.9, 0.36)
    assert p.theta == 0.5 and p.omega0 == 1.0
    # Section 5.1: termination tolerance and time limit
    assert p.tol == 1e-4 and p.time_limit_s == 3600.0
    assert p.precision == P.OT_PREC_FP32 and p.kkt_mode == 0 and p.restart_rule == 0
    assert p.engine == 0          # small instances resident, large ones on the whole GPU
    assert p.verify_retries == 8


def _dense(m, n):
    f = np.full(m, 1.0 / m)
    g = np.full(n, 1.0 / n)
    return f, g, np.zeros((m, n))


@pytest.mark.parametrize("case", ["m0", "n0", "tol", "ldc", "rows", "vec", "grid", "kind",
                                  "dim", "prec", "engine", "retries", "trace"])
def test_invalid_problems_rejected_before_device_work(case):
    f, g, C = _dense(4, 5)
    kw = {}
    pr = P.problem(P.OT_COST_DENSE, 4, 5, f, g, C=C)
    if case == "m0":
        pr = P.problem(P.OT_COST_DENSE, 0, 5, f, g, C=C)
    elif case == "n0":
        pr = P.problem(P.OT_COST_DENSE, 4, 0, f, g, C=C)
    elif case == "tol":
        kw["tol"] = 0.0
    elif case == "ldc":
        pr = P.problem(P.OT_COST_DENSE, 4, 5, f, g, C=C, ldc=3)
    elif case == "rows":
        kw["tile_rows"] = 24
    elif case == "vec":
        kw["tile_vec"] = 3
    elif case == "grid":
        pr = P.problem(P.OT_COST_GRID_SQEUCLID, 4, 5, f, g, side=2)
    elif case == "kind":
        pr = P.problem(7, 4, 5, f, g, C=C)
    elif case == "dim":
        x = np.zeros((4, 4))
        pr = P.problem(P.OT_COST_POINTS_SQEUCLID, 4, 5, f, g, x=x, y=np.zeros((5, 4)))
    elif case == "prec":
        kw["precision"] = 7
    elif case == "engine":
        kw["engine"] = 3
    elif case == "retries":
        kw["verify_retries"] = -1
    elif case == "trace":
        pr = P.problem(P.OT_COST_DENSE, 4, 5, f, g, C=C, trace_cap=4)
        pr.raw.trace_cap = -1
    st, _ = P.ot_solve(pr, P.params(**kw))
    assert st == P.OT_ERR_INVALID, (case, st, P.ot_last_error())
    assert P.ot_last_error()


def test_workspace_size_scales_with_precision_and_cost_storage():
    f, g, C = _dense(100, 300)
    pr = P.problem(P.OT_COST_DENSE, 100, 300, f, g, C=C)
    w32 = P.ot_workspace_size(pr, P.params(precision=P.OT_PREC_FP32))
    w64 = P.ot_workspace_size(pr, P.params(precision=P.OT_PREC_FP64))
    mat32 = 112 * 320 * 4          # rows padded to 16, columns to 64
    assert w32 >= 5 * mat32 and w64 >= 10 * mat32 and w64 > w32
    x = np.zeros((100, 2))
    y = np.zeros((300, 2))
    regen = P.problem(P.OT_COST_POINTS_SQEUCLID, 100, 300, f, g, x=x, y=y, store=0)
    stored = P.problem(P.OT_COST_POINTS_SQEUCLID, 100, 300, f, g, x=x, y=y, store=1)
    assert P.ot_workspace_size(stored, P.params()) - P.ot_workspace_size(regen, P.params()) >= mat32


def test_server_rejects_invalid_configuration_without_device_work():
    st, h = P.ot_server_create(1 << 10, max_active=4)
    assert st == P.OT_ERR_INVALID
    st, h = P.ot_server_create(1 << 30, max_active=0)
    assert st == P.OT_ERR_INVALID
    st, h = P.ot_server_create(1 << 30, max_active=4, prm=P.params(tol=-1.0))
    assert st == P.OT_ERR_INVALID


def test_round_rejects_invalid_arguments_without_device_work():
    f, g, C = _dense(4, 5)
    pr = P.problem(P.OT_COST_DENSE, 4, 5, f, g, C=C)
    X = np.zeros((4, 5))
    u = np.zeros(4)
    st, _ = P.ot_round(pr, P.OT_PREC_FP64, None, u)
    assert st == P.OT_ERR_INVALID
    st, _ = P.ot_round(pr, 7, X, u)
    assert st == P.OT_ERR_INVALID
    bad = P.problem(P.OT_COST_DENSE, 4, 5, f * 2.0, g, C=C)
    st, _ = P.ot_round(bad, P.OT_PREC_FP64, X, u)
    assert st == P.OT_ERR_INVALID
