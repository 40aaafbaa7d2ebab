"""Write the stored oracle values used by the GPU parity tests.

Calls only the FP64 oracle (oracle/) on the seeded workload generators; nothing here
comes from the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py            # every file
    python tests/golden/make_golden.py config3    # one of them

config2_oracle.json: the 32x32 blob grids of seed 100 (m = n = 1024) at tol 1e-6 and 1e-9.
config3_oracle.json: the 64x64 blob grids of seed 200 (m = n = 4096, the benchmark
workload) at tol 1e-6 and 1e-8, with the certified bracket of the tol-1e-8 plan (Algorithm
3 rounding for the upper bound, the c-transform of the returned row duals for the lower
one).  About 10 oracle iterations per second on 8 host cores at this size, so the file
takes tens of minutes to write.
"""
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import generators as gen  # noqa: E402


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def _solve_levels(inst, tols, out, path, bracket_at=None):
    C = inst.dense_cost()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    out["host"] = {"cpu_model": _cpu_model(), "threads": threads}
    for tol in tols:
        t = time.time()
        X, p, q, r, _ = oracle.solve(C, inst.f, inst.g, tol=tol, max_iters=1000000)
        assert r["status"] == 0
        key = f"tol{tol:g}"
        out[f"objective_{key}"] = r["objective"]
        out[f"rel_kkt_{key}"] = r["rel_kkt"]
        out[f"rel_primal_{key}"] = r["rel_primal"]
        out[f"iterations_{key}"] = r["iterations"]
        out[f"passes_{key}"] = r["passes"]
        out[f"restarts_{key}"] = r["restarts"]
        out[f"seconds_{key}"] = round(time.time() - t, 1)
        if bracket_at is not None and tol == bracket_at:
            Xf = oracle.round_plan(inst.f, inst.g, X)
            out[f"upper_{key}"] = float((C * Xf).sum())
            out[f"lower_{key}"] = oracle.dual_lower_bound(C, inst.f, inst.g, p)
        print(key, r["iterations"], r["objective"], f"{time.time() - t:.1f}s", flush=True)
        with open(path, "w") as fh:   # after every level, so a long run keeps what it has
            json.dump(out, fh, indent=1)
    return out


def config2():
    inst = gen.config_instance(2, 0)   # 32x32 blob images (seed 100), m = n = 1024
    out = {"workload": "config_instance(2, 0): two 32x32 blob histograms, seed 100, "
                       "squared pixel distance / (2*31^2)", "m": inst.m, "n": inst.n}
    return _solve_levels(inst, (1e-6, 1e-9), out, os.path.join(HERE, "config2_oracle.json"))


def config3():
    inst = gen.config_instance(3, 0)   # 64x64 blob images (seed 200), m = n = 4096
    out = {"workload": "config_instance(3, 0): two 64x64 blob histograms, seed 200, "
                       "squared pixel distance / (2*63^2)", "m": inst.m, "n": inst.n}
    return _solve_levels(inst, (1e-6, 1e-8), out, os.path.join(HERE, "config3_oracle.json"),
                         bracket_at=1e-8)


if __name__ == "__main__":
    which = sys.argv[1:] or ["config2", "config3"]
    for name in which:
        {"config2": config2, "config3": config3}[name]()
