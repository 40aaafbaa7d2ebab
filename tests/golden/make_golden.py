"""Write the stored oracle values used by the GPU parity tests.

Calls only the FP64 oracle (oracle/) on the seeded workload generators; nothing here
comes from the HIP path.  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import generators as gen  # noqa: E402


def config2():
    inst = gen.config_instance(2, 0)   # 32x32 blob images (seed 100), m = n = 1024
    C = inst.dense_cost()
    out = {"workload": "config_instance(2, 0): two 32x32 blob histograms, seed 100, "
                       "squared pixel distance / (2*31^2)", "m": inst.m, "n": inst.n}
    for tol in (1e-6, 1e-9):
        t = time.time()
        _, _, _, r, _ = oracle.solve(C, inst.f, inst.g, tol=tol, max_iters=1000000)
        assert r["status"] == 0
        key = f"tol{tol:g}"
        out[f"objective_{key}"] = r["objective"]
        out[f"rel_kkt_{key}"] = r["rel_kkt"]
        out[f"iterations_{key}"] = r["iterations"]
        print(key, r["iterations"], r["objective"], f"{time.time() - t:.1f}s", flush=True)
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "config2_oracle.json"), "w") as fh:
        json.dump(config2(), fh, indent=1)
