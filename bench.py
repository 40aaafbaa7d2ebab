"""Benchmark: restarted PDHG optimal transport on one MI355X.

Workload (m = n = 4096): two 64 x 64 blob-histogram images (seed 200; five Gaussian blobs
each, floor 1e-3, normalised), squared pixel distance scaled to max 1, regenerated inside
the streaming kernel; FP32 plan/average streams with FP64 duals, sums and control; solved
to relative KKT 1e-6.  One timed step is one complete solve (every iteration of it runs
the whole hot path: primal step, sums, dual step, averaging, KKT, restart and step-size
checks).  `value` is accepted PDHG iterations per second over the timed solves.

Also reported: time to 1e-4 and 1e-6, the stored-FP32-cost and plain-FP64 forms, the
streaming kernel against the HBM roofline (durations from HIP events around every pass
launch of one profiled solve), and the FP64 CPU oracle timed on a bounded sample.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-rel-KKT 1e-6 & PDHG iter/s (HBM GB/s) at m=n=4096; p50/p99 batched")
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2407_19689_amd", "csrc", "pdot_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_grid4096_fp32_traffic.md")
COPY_BYTES = 1 << 30          # the calibration copy moves 1 GiB each way


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def gpu_solve(P, inst, tol, precision, store, profile=0):
    import torch
    prm = P.params(tol=tol, precision=precision, time_limit_s=600.0, profile=profile)
    pr, out = P.problem_from_instance(inst, precision=precision, store=store, want_plan=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    st, res = P.ot_solve(pr, prm)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    if st not in (P.OT_OK,):
        raise RuntimeError(f"solve failed: {P.STATUS_NAMES.get(st)} {P.ot_last_error()}")
    return dt, res.as_dict()


def kernel_sha():
    import hashlib
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def traffic_probe():
    """Workload for the two counter runs (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE): a
    plain 1 GiB device copy (calibration) and 300 iterations of the benchmark solve."""
    import torch
    import paper_2407_19689_amd as P
    from workloads import generators as gen
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    inst = gen.grid_pair(200, 64)
    prm = P.params(tol=1e-12, precision=P.OT_PREC_FP32, max_iters=300, time_limit_s=60.0)
    pr, _ = P.problem_from_instance(inst, precision=P.OT_PREC_FP32, want_plan=False)
    st, r = P.ot_solve(pr, prm)
    torch.cuda.synchronize()
    launches = sum(r.mode_passes)
    print(json.dumps({"probe": "traffic", "launches": launches,
                      "algorithmic_bytes_per_launch": r.pass_bytes / launches,
                      "mode_passes": list(r.mode_passes)}), flush=True)


def summarize_traffic(fetch_dir, write_dir, probe_log):
    """Per-launch HBM traffic of the streaming pass from the two counter runs, each scaled
    by the counter's reading for the 1 GiB copy; writes the traffic summary in profiles/."""
    import csv
    import glob

    def per_dispatch(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        vals = {}
        for row in csv.DictReader(open(f)):
            if row.get("Counter_Name") != counter:
                continue
            key = (row["Dispatch_Id"], row["Kernel_Name"])
            vals[key] = vals.get(key, 0.0) + float(row["Counter_Value"])
        copy = [v for (i, k), v in vals.items() if "copy" in k.lower() or "elementwise" in k.lower()]
        kpass = [v for (i, k), v in vals.items() if "k_pass" in k]
        return max(copy), sum(kpass) / len(kpass), len(kpass)

    probe = [json.loads(x) for x in open(probe_log) if x.startswith('{"probe"')][0]
    fc, fp, nf = per_dispatch(fetch_dir, "FETCH_SIZE")
    wc, wp, nw = per_dispatch(write_dir, "WRITE_SIZE")
    kf, kw = COPY_BYTES / fc, COPY_BYTES / wc          # bytes per counter unit
    traffic = fp * kf + wp * kw
    algo = probe["algorithmic_bytes_per_launch"]
    lines = [
        "# k_pass (m=n=4096 grid, FP32 plan, cost regenerated): HBM traffic per launch",
        "",
        "Counters: `FETCH_SIZE` and `WRITE_SIZE` (KiB per dispatch), each in its own run:",
        "",
        "    rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o fetch -- python3 bench.py --traffic-probe",
        "    rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o write -- python3 bench.py --traffic-probe",
        "    python3 bench.py --summarize-traffic gpurun_out/pmc_fetch gpurun_out/pmc_write gpurun_out/traffic_probe.log",
        "",
        "Calibration: a plain 1 GiB device copy reads {:.0f} and writes {:.0f} counter units,".format(fc, wc),
        "so one unit is {:.1f} read bytes and {:.1f} written bytes.".format(kf, kw),
        "",
        "| quantity | per k_pass launch |",
        "|---|---|",
        "| FETCH_SIZE (units, mean of {} dispatches) | {:.0f} |".format(nf, fp),
        "| WRITE_SIZE (units, mean of {} dispatches) | {:.0f} |".format(nw, wp),
        "| read bytes (scaled) | {:.4g} |".format(fp * kf),
        "| written bytes (scaled) | {:.4g} |".format(wp * kw),
        "| traffic (read + written) | {:.4g} |".format(traffic),
        "| algorithmic bytes (same launch mix) | {:.4g} |".format(algo),
        "| traffic / algorithmic | {:.3f} |".format(traffic / algo),
        "",
        "traffic_bytes_per_launch: {:.0f}".format(traffic),
        "algorithmic_bytes_per_launch: {:.0f}".format(algo),
        "kernel_source_sha256: {}".format(kernel_sha()),
    ]
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def stored_traffic():
    """Traffic per launch from the committed counter summary, or None when the kernel
    source changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith(("#", "|", " ")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_sha():
        return None
    return float(vals["traffic_bytes_per_launch"]), float(vals["algorithmic_bytes_per_launch"])


def cpu_baseline(inst, budget_s=15.0):
    """The FP64 oracle on the host cores: PDHG iterations/s over the first iterations of
    the same instance (a bounded sample; the full solve would take hours)."""
    import numpy as np
    import oracle
    C = inst.dense_cost()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    # calibrate the per-iteration time (a 6-iteration run minus a 1-iteration run, which
    # removes the set-up), then run about budget_s of work
    t = time.perf_counter()
    oracle.solve(C, inst.f, inst.g, tol=1e-12, max_iters=1, nthreads=threads)
    t1 = time.perf_counter() - t
    t = time.perf_counter()
    oracle.solve(C, inst.f, inst.g, tol=1e-12, max_iters=6, nthreads=threads)
    per = max((time.perf_counter() - t - t1) / 5.0, 1e-6)
    iters = max(2, int(budget_s / per))
    t = time.perf_counter()
    _, _, _, res, _ = oracle.solve(C, inst.f, inst.g, tol=1e-12, max_iters=iters, nthreads=threads)
    dt = time.perf_counter() - t
    del C
    return {"value": res["iterations"] / dt, "unit": "iter/s", "cores": threads, "kind": "oracle",
            "sample": f"first {res['iterations']} PDHG iterations (FP64, dense C) of the m=n=4096 "
                      f"grid instance, {dt:.1f} s on {threads} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run the workload of the counter runs (see profiles/)")
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "PROBE_LOG"))
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic)
        return
    if args.traffic_probe:
        traffic_probe()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(instances shard across GPUs without communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2407_19689_amd as P
    from workloads import generators as gen

    torch.cuda.set_device(0)
    inst = gen.grid_pair(200, 64, tol=args.tol)
    FP32, FP64 = P.OT_PREC_FP32, P.OT_PREC_FP64

    for w in range(args.warmup):
        dt, r = gpu_solve(P, inst, args.tol, FP32, 0)
        log(f"warmup {w}: {dt:.3f} s, {r['iterations']} iterations")
    torch.cuda.synchronize()
    times, iters, last = [], [], None
    t0 = time.perf_counter()
    for k in range(args.steps):
        dt, r = gpu_solve(P, inst, args.tol, FP32, 0)
        times.append(dt)
        iters.append(r["iterations"])
        last = r
        log(f"step {k}: {dt:.3f} s, {r['iterations']} iterations, rel_kkt {r['rel_kkt']:.3e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    value = sum(iters) / sum(times)

    dt4, r4 = gpu_solve(P, inst, 1e-4, FP32, 0)
    log(f"tol 1e-4: {dt4:.3f} s, {r4['iterations']} iterations")

    # streaming kernel vs HBM roofline: HIP events around every pass launch of one solve
    dtp, rp = gpu_solve(P, inst, args.tol, FP32, 0, profile=1)
    launches = sum(rp["mode_passes"])
    avg_ms = rp["pass_ms"] / max(launches, 1)
    avg_bytes = rp["pass_bytes"] / max(launches, 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    log(f"profiled solve: {launches} pass launches, avg {avg_ms * 1e3:.2f} us, "
        f"{avg_bytes / 1e6:.1f} MB algorithmic, {achieved:.0f} GB/s; combine avg "
        f"{rp['combine_ms'] / max(launches, 1) * 1e3:.2f} us")
    st_tr = stored_traffic()
    traffic = None
    if st_tr is not None:
        # traffic measured per launch of the counter probe's launch mix, scaled to this mix
        traffic = round(st_tr[0] / st_tr[1] * avg_bytes)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_pass<float,4,grid-sqeuclid>", "avg_launch_us": round(avg_ms * 1e3, 3),
            "algorithmic_bytes_per_launch": round(avg_bytes), "launches": launches,
            "passes_by_kind": {"init": rp["mode_passes"][1], "trial": rp["mode_passes"][2],
                               "full": rp["mode_passes"][3], "restart": rp["mode_passes"][4],
                               "verify": rp["mode_passes"][5]}}

    forms = {}
    if not args.no_forms:
        for name, prec, store in (("fp32_stored_cost", FP32, 1), ("fp64_regenerated_cost", FP64, 0),
                                  ("fp64_stored_cost", FP64, 1)):
            dtf, rf = gpu_solve(P, inst, args.tol, prec, store)
            forms[name] = {"seconds": round(dtf, 4), "iterations": rf["iterations"],
                           "iter_per_s": round(rf["iterations"] / dtf, 1),
                           "objective": rf["objective"], "rel_kkt": rf["rel_kkt"]}
            log(f"form {name}: {dtf:.3f} s, {rf['iterations']} iterations")

    cpu = None if args.no_cpu else cpu_baseline(inst)

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / max(args.steps, 1), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage_dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "two 64x64 blob-histogram images (seed 200), m=n=4096, squared "
                               "pixel distance / (2*63^2) regenerated in-kernel, FP32 plan and "
                               "average streams, FP64 duals/sums/control, rel-KKT tol 1e-6",
                   "m": 4096, "n": 4096, "tol": args.tol},
        "time_to_tol_s": {"1e-6": round(sum(times) / len(times), 4), "1e-4": round(dt4, 4)},
        "iterations": {"1e-6": last["iterations"], "1e-4": r4["iterations"]},
        "restarts": last["restarts"],
        "passes": last["passes"],
        "objective": last["objective"],
        "rel_kkt": last["rel_kkt"],
        "roofline": roof,
        "forms": forms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
