"""Throughput of the MOL^T wave solver on one MI355X.

Workload (default): 2D ADI, order 2P = 4 (P = 2), unit square, 4096 x 4096
nodes, homogeneous Dirichlet, CFL = 2, FP32, initial data = 8 Gaussian pulses
(width 0.02, seeded).  One step = one pass of the whole hot path: every
directional sweep of the stage schedule, the ADI compositions and the time
update.  The timed region replays K steps (hipGraph) with the fields resident
in HBM, bracketed by device synchronisation and timed with HIP events on the
library's stream.

The JSON line also carries
* roofline: the dominant kernel's algorithmic bytes per launch over its mean
  duration (HIP events around each launch of one step), against 8 TB/s;
* cpu_baseline: the FP64 CPU oracle on one step of the same grid (the host's
  cores), in the same unit;
* also: the 1024^2 P = 2 workload (500 steps, FP64 and FP32).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mpoint-updates/s & %HBM roofline (2D ADI P=2); p50/p99 served latency"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("molt_kernels.hip", "molt_plan.cpp"):
        with open(os.path.join(ROOT, "paper_1308_3214_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_tag: str):
    """Measured HBM bytes per launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    ent = d.get("kernels", {}).get(kernel_tag)
    return None if ent is None else ent.get("bytes_per_launch")


def run_gpu(n, P, cfl, dtype, steps, warmup, seed=1):
    import torch
    from paper_1308_3214_amd import molt
    from paper_1308_3214_amd import workloads as W

    h = 1.0 / (n - 1)
    plan = molt.Plan((n, n), h, molt.DIRICHLET, P=P, cfl=cfl, dtype=dtype)
    td = torch.float64 if dtype == "f64" else torch.float32
    u0 = torch.tensor(W.gaussian_pulses_2d(n, seed=seed), dtype=td, device="cuda")
    u1 = torch.empty_like(u0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.start(u0, u1)
        plan.solve(u0, u1, warmup)           # also captures the graph
        stream.synchronize()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.solve(u0, u1, steps)
        e1.record(stream)
        stream.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert torch.isfinite(u1).all().item(), "non-finite field"
    # per-kernel breakdown of one step (events around every launch)
    scratch = torch.empty_like(u0)
    with torch.cuda.stream(stream):
        kern = plan.profile_step(u0, u1, scratch, reps=max(3, min(20, steps // 5)))
    torch.cuda.synchronize()
    info = plan.info
    plan.close()
    return ms, kern, info


def serve(count=256, rate_hz=50.0, seed=1, budget=2 << 30, nstreams=4, burst=False, steps=100):
    """The serving workload: a Poisson stream of independent FP32 requests
    (n log-uniform in [128, 2048], P in {1, 2, 3}, CFL in [1, 4], 100 steps,
    4 Gaussian pulses) through the request server with a device budget.
    Latency = scheduled arrival -> completion seen by the polling loop."""
    import numpy as np
    import torch
    from paper_1308_3214_amd import molt
    from paper_1308_3214_amd import workloads as W
    reqs = W.request_stream(count, rate_hz, seed, steps=steps, burst=burst)
    # initial fields in pinned host memory, made before the clock starts
    inits = [torch.from_numpy(W.request_initial(r).astype(np.float32)).pin_memory() for r in reqs]
    srv = molt.Server(budget, nstreams)
    arrival, done_t, rid_of = {}, {}, {}
    t0 = time.perf_counter()
    i = 0
    while len(done_t) < count:
        now = time.perf_counter() - t0
        while i < count and reqs[i].arrival_s <= now:
            r = reqs[i]
            rid = srv.submit(inits[i], (r.n, r.n), 1.0 / (r.n - 1), r.steps, P=r.P, cfl=r.cfl,
                             dtype="f32")
            arrival[rid] = r.arrival_s
            rid_of[rid] = i
            i += 1
        got = srv.poll()
        tn = time.perf_counter() - t0
        for rid in got:
            done_t[rid] = tn
            srv.result(rid)                 # back to the client (host)
        if not got:
            time.sleep(50e-6)
        if tn > 300:
            raise RuntimeError("serving run did not finish")
    st = srv.stats()
    srv.close()
    lat = np.array([done_t[k] - arrival[k] for k in done_t]) * 1e3
    pts = float(sum(r.n * r.n * r.steps for r in reqs))
    span = max(done_t.values()) - min(r.arrival_s for r in reqs)
    return {"requests": count, "rate_hz": None if burst else rate_hz, "burst": burst,
            "budget_bytes": budget, "streams": nstreams,
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3),
            "Mpoint-updates/s": round(pts / span / 1e6, 1),
            "span_s": round(span, 3), "peak_bytes": st["bytes_peak"]}


def cpu_baseline(n, P, cfl, nsteps=1, seed=1):
    import numpy as np
    import oracle
    from paper_1308_3214_amd import workloads as W
    h = 1.0 / (n - 1)
    b = oracle.beta_max(P)
    pb = oracle.Problem((n, n), h, oracle.DIRICHLET, b / (cfl * h))
    u0 = W.gaussian_pulses_2d(n, seed=seed)
    u1 = u0.copy()
    t = time.perf_counter()
    pb.run(u0, u1, nsteps, P, b)
    dt = time.perf_counter() - t
    return {"value": n * n * nsteps / dt / 1e6, "unit": "Mpoint-updates/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d step(s) of the %dx%d P=%d FP64 workload, %.1f s" % (nsteps, n, n, P, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--P", type=int, default=2)
    ap.add_argument("--cfl", type=float, default=2.0)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-also", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver is built and measured on a single "
              "MI355X (multi-GPU slab decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    n, P = args.n, args.P
    ms, kern, info = run_gpu(n, P, args.cfl, args.dtype, args.steps, args.warmup)
    ms_step = ms / args.steps
    points = n * n
    value = points / (ms_step * 1e-3) / 1e6
    # dominant kernel
    dom = max(range(len(kern)), key=lambda i: kern[i]["ms"])
    k = kern[dom]
    achieved = k["bytes"] / (k["ms"] * 1e-3) / 1e9
    tag = "%s_sweep_k%d" % (k["dir"], dom)
    traffic = traffic_for(tag)
    step_gbs = info["bytes_per_step"] / (ms_step * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpoint-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "2D ADI P=%d, %dx%d unit square, Dirichlet, CFL %g, %s, 8 Gaussian "
                               "pulses (sigma 0.02, seed 1)" % (P, n, n, args.cfl, args.dtype),
                   "grid": [n, n], "P": P, "cfl": args.cfl, "beta": info["beta"],
                   "nu": info["nu"][0], "kernels_per_step": info["kernels_per_step"],
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": tag,
                     "kernel_ms": round(k["ms"], 5), "kernel_bytes": k["bytes"]},
        "step_bytes": info["bytes_per_step"],
        "step_hbm_frac": round(step_gbs / HBM_PEAK_GBS, 4),
        "kernels": [{"dir": x["dir"], "sweeps": x["sweeps"], "ms": round(x["ms"], 5),
                     "GB/s": round(x["bytes"] / (x["ms"] * 1e-3) / 1e9, 1)} for x in kern],
    }
    if not args.no_also:
        also = {}
        for dt in ("f64", "f32"):
            ms2, _, inf2 = run_gpu(1024, 2, 2.0, dt, 500, 10)
            also["1024x1024_P2_%s_500steps" % dt] = {
                "Mpoint-updates/s": round(1024 * 1024 * 500 / (ms2 * 1e-3) / 1e6, 2),
                "ms_per_step": round(ms2 / 500, 5)}
        fp64 = run_gpu(n, P, args.cfl, "f64", max(20, args.steps // 4), 5)
        also["%dx%d_P%d_f64" % (n, n, P)] = {
            "Mpoint-updates/s": round(points / (fp64[0] / max(20, args.steps // 4) * 1e-3) / 1e6, 2)}
        out["also"] = also
    if not args.no_serve:
        out["serving"] = {"poisson": serve(), "burst": serve(burst=True)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, P, args.cfl, 1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
