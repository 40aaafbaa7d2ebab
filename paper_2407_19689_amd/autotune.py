"""Tile-shape autotuner for the streaming pass.

For each cost kind (Euclidean and squared-Euclidean point clouds; images under the
squared-Euclidean, l1, l2 and l-infinity ground costs) and precision (FP32 and FP64
plans), representative instances on a grid of size buckets
(m, n = powers of two) are solved for a fixed number of iterations with every candidate
tile shape (columns per lane VEC in {1, 2, 4}, rows per tile in {16, ..., 256}) in
profiling mode; the shape with the smallest measured slot time (streaming pass plus
combine) wins.  The results are cached as JSON next to this file, keyed by
architecture, precision, cost kind and bucket; `tiles_for` returns the cached choice for
the nearest bucket (or (0, 0), which selects the library's built-in heuristic).

The tile shape only changes the order of the deterministic reductions, never the method,
so every choice gives a valid solve; the batch and the server take the per-instance
choice through `ot_problem.tile_vec / tile_rows`.

Usage (on the GPU):
    python -m paper_2407_19689_amd.autotune [--quick] [--kinds K1,K2] [--precisions 1,0]
"""
import argparse
import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_gfx950.json")
GRID_KINDS = ("grid_sqeuclid", "grid_l1", "grid_l2", "grid_linf")
KINDS = ("points_euclid", "points_sqeuclid") + GRID_KINDS
# size buckets (log2 m = log2 n range) per cost kind: Euclidean point clouds for batches of
# 32..2048 points, squared-Euclidean clouds and square images for requests up to 16384
EXPS = {"points_euclid": range(5, 12), "points_sqeuclid": range(6, 15)}
EXPS.update({k: range(6, 15, 2) for k in GRID_KINDS})


def bucket(m, n):
    return int(round(math.log2(max(m, 1)))), int(round(math.log2(max(n, 1))))


def _key(precision, kind, bm, bn):
    return f"gfx950/p{precision}/{kind}/{bm}x{bn}"


_cache = None


def load_cache():
    global _cache
    if _cache is None:
        _cache = json.load(open(CACHE)) if os.path.exists(CACHE) else {}
    return _cache


def tiles_for(m, n, precision, kind, shared=False):
    """(vec, rows) from the cache for the nearest tuned bucket, else (0, 0).

    The cache holds the shapes measured best for an instance running alone, where narrow
    lanes (1-2 columns) buy more tiles to fill the GPU.  With shared=True (many instances
    solved together, which fill the GPU between them) the lane is the widest the instance's
    n allows (fewer per-row instructions per byte) and the rows stay the tuned ones: on the
    256-instance batch that was 5 % shorter makespan and 8 % lower completion p50."""
    v, r = _tuned(m, n, precision, kind)
    if shared:
        v = 4 if n >= 256 else (2 if n >= 128 else 1)
    return v, r


def _tuned(m, n, precision, kind):
    cache = load_cache()
    bm, bn = bucket(m, n)
    best, dist = (0, 0), None
    prefix = f"gfx950/p{precision}/{kind}/"
    for k, v in cache.items():
        if not k.startswith(prefix):
            continue
        km, kn = (int(t) for t in k[len(prefix):].split("x"))
        d = abs(km - bm) + abs(kn - bn)
        if dist is None or d < dist:
            best, dist = (v["vec"], v["rows"]), d
    return best


def _instance(kind, m, n, seed):
    from workloads import generators as gen
    if kind == "points_euclid":
        return gen.gmm_euclid(seed, m, n)
    if kind == "points_sqeuclid":
        return gen.points_sqeuclid(seed, m, n)
    side = int(round(math.sqrt(m)))
    return gen.grid_pair(seed, side, kind=kind)


def measure(inst, precision, vec, rows, iters):
    import torch
    import paper_2407_19689_amd as P
    prm = P.params(tol=1e-12, precision=precision, max_iters=iters, profile=1, tile_vec=vec,
                   tile_rows=rows, time_limit_s=30.0)
    pr, _ = P.problem_from_instance(inst, precision=precision, want_plan=False)
    st, r = P.ot_solve(pr, prm)
    torch.cuda.synchronize()
    launches = sum(r.mode_passes)
    if st not in (P.OT_OK, P.OT_NOT_CONVERGED) or launches == 0 or r.pass_ms <= 0.0:
        return None
    return (r.pass_ms + r.combine_ms) / launches


def tune(kinds=KINDS, precision=1, quick=False, iters=60, verbose=True, out=None):
    # start from the output file when it exists (several calls add to one file)
    cache = dict(json.load(open(out)) if out and os.path.exists(out) else load_cache())
    for kind in kinds:
        exps = list(EXPS[kind])[::2] if quick and kind not in GRID_KINDS else EXPS[kind]
        for em in exps:
            for en in exps:
                if kind in GRID_KINDS and em != en:
                    continue              # square images only: m = n = side^2
                m, n = 2 ** em, 2 ** en
                inst = _instance(kind, m, n, seed=em * 100 + en)
                m, n = inst.m, inst.n
                best = None
                for vec in (1, 2, 4):
                    if 64 * vec > 2 * n and vec > 1:
                        continue
                    for rows in (16, 32, 64, 128, 256):
                        if rows > max(16, 2 * m):
                            continue
                        t = measure(inst, precision, vec, rows, iters)
                        if t is not None and (best is None or t < best[0]):
                            best = (t, vec, rows)
                if best is None:
                    continue
                cache[_key(precision, kind, *bucket(m, n))] = {
                    "vec": best[1], "rows": best[2], "slot_ms": round(best[0], 5), "m": m, "n": n}
                if verbose:
                    print(f"p{precision} {kind} m={m} n={n}: vec={best[1]} rows={best[2]} "
                          f"slot {best[0] * 1e3:.1f} us", flush=True)
        with open(out or CACHE, "w") as fh:   # after every kind: a cut-off run keeps its results
            json.dump(cache, fh, indent=1, sort_keys=True)
    return cache


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer buckets and iterations")
    ap.add_argument("--kinds", default=",".join(KINDS))
    ap.add_argument("--precisions", default="1,0", help="1: FP32 plan, 0: FP64 plan")
    ap.add_argument("--out", default=None, help="write the cache here instead of next to the module")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    t = time.time()
    for prec in (int(p) for p in args.precisions.split(",")):
        tune(kinds=args.kinds.split(","), precision=prec, quick=args.quick,
             iters=40 if args.quick else 60, out=args.out)
    print(f"autotune done in {time.time() - t:.1f} s -> {args.out or CACHE}", flush=True)


if __name__ == "__main__":
    main()
