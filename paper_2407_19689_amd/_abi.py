"""ctypes mirror of ``include/pdot.h``: structures, enums and the library loader.

Argument marshalling only; every step of the solver runs in the HIP library.  Loading
fails loudly when ``libpdot.so`` has not been built -- there is no fallback path.
"""
import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PDOT_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("PDOT_LIBRARY") or os.path.join(HERE, "libpdot.so")

# ot_status
OT_OK = 0
OT_ERR_INVALID = 1
OT_ERR_OOM = 2
OT_ERR_DEVICE = 3
OT_NOT_CONVERGED = 4
OT_ERR_NUMERIC = 5
OT_ERR_BUSY = 6
STATUS_NAMES = {0: "OK", 1: "ERR_INVALID", 2: "ERR_OOM", 3: "ERR_DEVICE", 4: "NOT_CONVERGED",
                5: "ERR_NUMERIC", 6: "ERR_BUSY"}

# ot_precision
OT_PREC_FP64 = 0
OT_PREC_FP32 = 1

# ot_cost_kind
OT_COST_DENSE = 0
OT_COST_POINTS_SQEUCLID = 1
OT_COST_POINTS_EUCLID = 2
OT_COST_GRID_SQEUCLID = 3
OT_COST_GRID_L1 = 4
OT_COST_GRID_L2 = 5
OT_COST_GRID_LINF = 6

# bytes of the static device array behind ot_solve_noalloc
OT_NOALLOC_MAX_BYTES = 128 << 20

_D = ct.POINTER(ct.c_double)


class OtCost(ct.Structure):
    _fields_ = [
        ("kind", ct.c_int32),
        ("dim", ct.c_int32),
        ("side", ct.c_int32),
        ("store", ct.c_int32),
        ("ldc", ct.c_int64),
        ("C", ct.c_void_p),
        ("x", ct.c_void_p),
        ("y", ct.c_void_p),
        ("scale", ct.c_double),
    ]


class OtTraceRec(ct.Structure):
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


class OtProblem(ct.Structure):
    _fields_ = [
        ("cost", OtCost),
        ("m", ct.c_int64),
        ("n", ct.c_int64),
        ("f", ct.c_void_p),
        ("g", ct.c_void_p),
        ("tol", ct.c_double),
        ("X_out", ct.c_void_p),
        ("u_out", ct.c_void_p),
        ("v_out", ct.c_void_p),
        ("tile_vec", ct.c_int32),
        ("tile_rows", ct.c_int32),
        ("trace", ct.c_void_p),
        ("trace_cap", ct.c_int64),
    ]


class OtParams(ct.Structure):
    _fields_ = [
        ("tol", ct.c_double),
        ("max_iters", ct.c_int64),
        ("max_passes", ct.c_int64),
        ("time_limit_s", ct.c_double),
        ("precision", ct.c_int32),
        ("kkt_mode", ct.c_int32),
        ("step_rule", ct.c_int32),
        ("restart_rule", ct.c_int32),
        ("avg_weighting", ct.c_int32),
        ("primal_weight_update", ct.c_int32),
        ("output", ct.c_int32),
        ("graph_slots", ct.c_int32),
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
        ("tile_vec", ct.c_int32),
        ("tile_rows", ct.c_int32),
        ("profile", ct.c_int32),
        ("engine", ct.c_int32),
        ("verify_retries", ct.c_int32),
        ("pad0", ct.c_int32),
    ]


class OtResult(ct.Structure):
    _fields_ = [
        ("status", ct.c_int32),
        ("returned_average", ct.c_int32),
        ("iterations", ct.c_int64),
        ("passes", ct.c_int64),
        ("restarts", ct.c_int64),
        ("kernel_passes", ct.c_int64),
        ("objective", ct.c_double),
        ("dual_objective", ct.c_double),
        ("rel_primal", ct.c_double),
        ("rel_dual", ct.c_double),
        ("rel_gap", ct.c_double),
        ("rel_kkt", ct.c_double),
        ("eta", ct.c_double),
        ("omega", ct.c_double),
        ("seconds", ct.c_double),
        ("mode_passes", ct.c_int64 * 7),
        ("pass_bytes", ct.c_double),
        ("pass_ms", ct.c_double),
        ("combine_ms", ct.c_double),
        ("verify_retries", ct.c_int64),
        ("kkt_estimate", ct.c_double),
        ("estimate_parts", ct.c_double * 3),
        ("estimate_objective", ct.c_double),
        ("avg_fold_passes", ct.c_int64),
        ("trace_len", ct.c_int64),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["mode_passes"] = list(self.mode_passes)
        d["estimate_parts"] = list(self.estimate_parts)
        return d


class OtBracket(ct.Structure):
    _fields_ = [
        ("upper", ct.c_double),
        ("lower", ct.c_double),
        ("l1_change", ct.c_double),
        ("marginal_l1", ct.c_double),
        ("feas_violation", ct.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OtServerCfg(ct.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ct.c_size_t),
        ("max_active", ct.c_int32),
        ("max_queue", ct.c_int32),
        ("block_ms", ct.c_double),
        ("params", OtParams),
    ]


class OtCompletion(ct.Structure):
    _fields_ = [
        ("ticket", ct.c_uint64),
        ("result", OtResult),
        ("t_submit", ct.c_double),
        ("t_admit", ct.c_double),
        ("t_done", ct.c_double),
    ]


class OtServerStats(ct.Structure):
    _fields_ = [
        ("submitted", ct.c_int64),
        ("admitted", ct.c_int64),
        ("completed", ct.c_int64),
        ("running", ct.c_int64),
        ("queued", ct.c_int64),
        ("arena_used", ct.c_int64),
        ("arena_peak", ct.c_int64),
        ("launches", ct.c_int64),
        ("max_running", ct.c_int64),
    ]


# Every symbol the header declares, with (restype, argtypes).
SIGNATURES = {
    "ot_params_default": (None, [ct.POINTER(OtParams)]),
    "ot_workspace_size": (ct.c_size_t, [ct.POINTER(OtProblem), ct.POINTER(OtParams)]),
    "ot_solve": (ct.c_int, [ct.POINTER(OtProblem), ct.POINTER(OtParams), ct.POINTER(OtResult),
                            ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "ot_solve_noalloc": (ct.c_int, [ct.POINTER(OtProblem), ct.POINTER(OtParams), ct.POINTER(OtResult),
                                    ct.c_void_p]),
    "ot_solve_batch": (ct.c_int, [ct.POINTER(OtProblem), ct.c_int32, ct.POINTER(OtParams),
                                  ct.POINTER(OtResult), ct.c_void_p]),
    "ot_round": (ct.c_int, [ct.POINTER(OtProblem), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                            ct.POINTER(OtBracket), ct.c_void_p]),
    "ot_server_create": (ct.c_int, [ct.POINTER(OtServerCfg), ct.POINTER(ct.c_void_p)]),
    "ot_server_submit": (ct.c_int, [ct.c_void_p, ct.POINTER(OtProblem), ct.POINTER(ct.c_uint64)]),
    "ot_server_poll": (ct.c_int, [ct.c_void_p, ct.POINTER(OtCompletion), ct.c_int32,
                                  ct.POINTER(ct.c_int32)]),
    "ot_server_drain": (ct.c_int, [ct.c_void_p, ct.c_double]),
    "ot_server_get_stats": (ct.c_int, [ct.c_void_p, ct.POINTER(OtServerStats)]),
    "ot_server_destroy": (ct.c_int, [ct.c_void_p]),
    "ot_last_error": (ct.c_char_p, []),
    "ot_version": (ct.c_char_p, []),
}

_lib = None


def load():
    """Load ``libpdot.so`` (raises if it is missing: build it with build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2407_19689_amd/build.py "
                           "(the solver has no CPU fallback)")
    lib = ct.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
