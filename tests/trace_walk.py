"""Decision-by-decision comparison of two control traces of restarted PDHG (Section 5).

A trace is a list of dicts, one per rejected step trial and one per accepted iteration,
with the keys of the oracle's records: pass, iter, accepted, restart, cand_avg, eta_used,
eta_bar, k_cur, k_avg, omega.

Two implementations that sum in different orders do not stay at the rounding level with
the adaptive step: the step bound's denominator dy^T A dx and the duality gap are
differences of nearly equal sums, and the step rule feeds the bound back into eta, so the
trajectories separate by roughly a factor 1000 every 60 iterations (from about 1e-15), and
once the separation reaches the margins of the comparisons the decisions may part.  So the
walk covers the prefix in which the traced scalars (eta used, omega, both KKT values)
still agree to drift_cap; over that prefix every decision (pass and iteration numbers,
accepted or rejected, restart and its condition, candidate side) must be identical, and
eta_bar must agree where it can decide anything.
"""
import math


def _rel(a, b):
    return abs(a - b) / abs(b) if b != 0 else abs(a)


def walk_traces(tr, tr_ref, drift_cap=1e-6):
    """Assert that tr follows tr_ref over their common prefix; return the compared
    entries of tr_ref."""
    compared = []
    for a, b in zip(tr, tr_ref):
        keys = ("eta_used", "omega") + (("k_cur", "k_avg") if b["accepted"] else ())
        if max(_rel(a[k], b[k]) for k in keys) > drift_cap:
            break
        for key in ("pass", "iter", "accepted", "restart", "cand_avg"):
            ka = key if key in a else key + "_"
            kb = key if key in b else key + "_"
            assert a[ka] == b[kb], (key, a, b)
        va, vb = a["eta_bar"], b["eta_bar"]
        if math.isinf(vb):
            assert math.isinf(va), (a, b)
        elif vb <= 10.0 * b["eta_used"]:
            assert _rel(va, vb) <= 100.0 * drift_cap, (a, b)
        else:   # far above the step in use it decides nothing; its denominator is noise
            assert va > 5.0 * b["eta_used"], (a, b)
        compared.append(b)
    return compared
