"""Autotuner for the sweep kernels' launch configurations.

For every kernel of a plan's solve step, times each valid configuration (tile
shape / line-to-wave mapping) with HIP events around the launch
(mol_profile_step) and keeps the fastest.  Results go to the tuning cache the
plan reads at creation (tune_cache.txt beside libmolt.so, or the file named by
MOLT_TUNE_CACHE): one line per (problem, kernel shape).

    python -m paper_1308_3214_amd.tune                  # default problem set
    python -m paper_1308_3214_amd.tune --n 4096 --P 2 --dtype f32
    python -m paper_1308_3214_amd.tune --n 4096 --P 2 --dtype f32 --cfl 100

The key of a kernel shape does not hold the CFL number; the sweeps of the
small-nu step (the L^{-1} form) carry their own key suffix, so tuning at a
large CFL adds entries beside those of CFL 2.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.txt")

# problems tuned by default: the 2D workloads of the benchmark and tests
DEFAULT_PROBLEMS = [
    dict(shape=(4096, 4096), P=2, dtype="f32"),
    dict(shape=(4096, 4096), P=2, dtype="f64"),
    dict(shape=(1024, 1024), P=2, dtype="f32"),
    dict(shape=(1024, 1024), P=2, dtype="f64"),
    dict(shape=(256, 256, 256), P=2, dtype="f32", bc=1),
]


def tune_problem(shape, P, dtype, cfl=2.0, reps=10, verbose=True, bc=0):
    import torch
    from . import molt
    nd = len(shape)
    h = 1.0 / shape[-1] if bc == 1 else 1.0 / (shape[-1] - 1)
    plan = molt.Plan(shape, h, bc, P=P, cfl=cfl, dtype=dtype)
    td = torch.float64 if dtype == "f64" else torch.float32
    a = torch.rand(shape, dtype=td, device="cuda")
    b = torch.rand(shape, dtype=td, device="cuda")
    c = torch.empty_like(a)
    nk = plan.info["kernels_per_step"]
    lines = {}
    report = []
    for k in range(nk):
        ids, cur = plan.kernel_configs(k)
        best = None
        times = {}
        for cfg in ids:
            plan.set_kernel_config(k, cfg)
            plan.profile_step(a, b, c, reps=2)          # warm
            ms = plan.profile_step(a, b, c, reps=reps)[k]["ms"]
            times[cfg] = ms
            if best is None or ms < times[best]:
                best = cfg
        plan.set_kernel_config(k, best)
        key = plan.tune_key(k)
        lines[key] = best
        report.append({"kernel": k, "key": key, "best": best, "default": cur,
                       "ms": {str(i): round(t, 5) for i, t in times.items()}})
        if verbose:
            print("  kernel %d: best cfg %d (%.4f ms), default %d (%.4f ms)"
                  % (k, best, times[best], cur, times.get(cur, float("nan"))), flush=True)
    plan.close()
    return lines, report


def write_cache(entries, path=DEFAULT_CACHE):
    old = {}
    if os.path.exists(path):
        for ln in open(path):
            ln = ln.rstrip("\n")
            if " | " in ln:
                key, cfg = ln.rsplit(" | ", 1)
                old[key] = cfg
    for k, v in entries.items():
        old[k] = str(v)
    with open(path, "w") as f:
        for k in sorted(old):
            f.write("%s | %s\n" % (k, old[k]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--P", type=int, default=2)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--ndim", type=int, default=2)
    ap.add_argument("--bc", type=int, default=0)
    ap.add_argument("--cfl", type=float, default=2.0)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--report", default="")
    args = ap.parse_args()
    probs = DEFAULT_PROBLEMS if args.n == 0 else [dict(shape=(args.n,) * args.ndim, P=args.P,
                                                        dtype=args.dtype, bc=args.bc, cfl=args.cfl)]
    allent, allrep = {}, []
    for pr in probs:
        print("tuning", pr, flush=True)
        ent, rep = tune_problem(pr["shape"], pr["P"], pr["dtype"], cfl=pr.get("cfl", 2.0),
                                bc=pr.get("bc", 0))
        allent.update(ent)
        allrep.append({"problem": {k: list(v) if isinstance(v, tuple) else v
                                   for k, v in pr.items()}, "kernels": rep})
    write_cache(allent, args.cache)
    if args.report:
        json.dump(allrep, open(args.report, "w"), indent=1)
    print("wrote", args.cache)


if __name__ == "__main__":
    sys.exit(main())
