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
    """Hash of the kernel and plan sources: counter data taken on other
    sources is not reported."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1308_3214_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_tag: str):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled
    by the copy calibration) from profiles/traffic.txt, if the counters were
    taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(p):
        return None
    src, found = None, None
    for line in open(p):
        f = line.split()
        if len(f) >= 2 and f[0] == "source_hash":
            src = f[1]
        elif len(f) >= 6 and f[0] == "kernel" and f[1] == kernel_tag:
            found = float(f[3]) + float(f[5])
    if src != kernel_source_hash():
        return None
    return found


def run_plan(shape, h, bc, P, cfl, dtype, u0, steps, warmup, profile=True, keep=None, reps=5, **kw):
    """Time `steps` steps of mol_solve after `warmup` untimed steps: the
    graphs a `steps`-step call replays are captured beforehand
    (mol_solve_prepare, nothing run), then `reps` calls of `steps` steps are
    timed one by one with HIP events on the library's stream, each bracketed
    by device synchronisation; returns the median call.  Optional per-kernel
    breakdown; `keep` (a list) receives the final field on the host."""
    import torch
    from paper_1308_3214_amd import molt

    plan = molt.Plan(shape, h, bc, P=P, cfl=cfl, dtype=dtype, **kw)
    td = torch.float64 if dtype == "f64" else torch.float32
    a = torch.tensor(u0, dtype=td, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.Stream()
    times = []
    with torch.cuda.stream(stream):
        plan.start(a, b)
        plan.solve(a, b, warmup)
        plan.solve_prepare(a, b, steps)
        for _ in range(reps):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            plan.solve(a, b, steps)
            e1.record(stream)
            stream.synchronize()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
    ms = sorted(times)[len(times) // 2]
    assert torch.isfinite(b).all().item(), "non-finite field"
    if keep is not None:
        keep.append(b.double().cpu().numpy())
    kern = None
    if profile:
        # per-kernel breakdown of one step (events around every launch)
        scratch = torch.empty_like(a)
        with torch.cuda.stream(stream):
            kern = plan.profile_step(a, b, scratch, reps=max(3, min(20, steps // 5)))
        torch.cuda.synchronize()
    info = dict(plan.info)
    info["rep_ms"] = [round(t, 4) for t in times]
    plan.close()
    return ms, kern, info


GOLDEN = os.path.join(ROOT, "tests", "golden")


def fixture_error(name, field):
    """Error of a field against a sampled oracle result under tests/golden/
    (written by tests/golden/make_long_runs.py, which calls only the oracle):
    relative L2 over the samples and the largest sampled error relative to
    max |u|."""
    import numpy as np
    idx, ref, mx = [], [], None
    path = os.path.join(GOLDEN, name + ".txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            a, b = line.split()
            if a == "maxabs":
                mx = float(b)
            elif a != "l2norm":
                idx.append(int(a))
                ref.append(float(b))
    idx, ref = np.array(idx), np.array(ref)
    g = np.asarray(field, dtype=np.float64).ravel()[idx]
    return {"vs": "80-bit oracle, %d sampled nodes (%s)" % (idx.size, name),
            "rel_L2": float("%.3e" % (np.linalg.norm(g - ref) / np.linalg.norm(ref))),
            "max_elem": float("%.3e" % (np.abs(g - ref).max() / mx))}


def solve_from_start(shape, h, bc, P, cfl, dtype, u0, nsteps, **kw):
    """u^nsteps from mol_start and nsteps - 1 steps of mol_solve (graph
    replay on a non-default stream), on the host."""
    import torch
    from paper_1308_3214_amd import molt
    plan = molt.Plan(shape, h, bc, P=P, cfl=cfl, dtype=dtype, **kw)
    td = torch.float64 if dtype == "f64" else torch.float32
    a = torch.tensor(u0, dtype=td, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.start(a, b)
        plan.solve(a, b, nsteps - 1)
    torch.cuda.synchronize()
    out = b.double().cpu().numpy()
    plan.close()
    return out


def run_gpu(n, P, cfl, dtype, steps, warmup, seed=1, keep=None, flags=0, reps=15):
    from paper_1308_3214_amd import workloads as W
    u0 = W.gaussian_pulses_2d(n, seed=seed)
    return run_plan((n, n), 1.0 / (n - 1), 0, P, cfl, dtype, u0, steps, warmup, keep=keep,
                    flags=flags, reps=reps)


def also_line(ms, steps, info, points):
    step_ms = ms / steps
    out = {"Mpoint-updates/s": round(points / (step_ms * 1e-3) / 1e6, 2),
           "ms_per_step": round(step_ms, 5),
           "model_hbm_frac": round(info["bytes_per_step"] / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if "rep_ms" in info:
        out["steps_per_rep"] = steps
        out["rep_ms"] = info["rep_ms"]
    return out


def cfl_lines(n, P, dtype, steps, warmup):
    """The A-stable regime: CFL 10, 100 and 1000 on the headline grid."""
    out = {}
    for cfl in (10.0, 100.0, 1000.0):
        msc, kc, infc = run_gpu(n, P, cfl, dtype, steps, warmup)
        lc = also_line(msc, steps, infc, n * n)
        lc["nu"] = round(infc["nu"][0], 6)
        lc["kernels"] = [{"dir": x["dir"], "sweeps": x["sweeps"], "ms": round(x["ms"], 5),
                          "GB/s": round(x["bytes"] / (x["ms"] * 1e-3) / 1e9, 1)} for x in kc]
        if n == 4096 and P == 2:
            from paper_1308_3214_amd import workloads as W
            u10 = solve_from_start((n, n), 1.0 / (n - 1), 0, P, cfl, dtype,
                                   W.gaussian_pulses_2d(n, seed=1), 10)
            lc["error_u10"] = fixture_error("adi4096_p2_cfl%d_10" % cfl, u10)
        out["%dx%d_P%d_%s_cfl%g" % (n, n, P, dtype, cfl)] = lc
    return out


def line1d_workload(steps=200, warmup=10):
    """1D, N = 1024, Dirichlet, P = 1, CFL 2, FP64, two sine modes with seeded
    amplitudes (the 1D configuration): one line of 1024 nodes per step."""
    from paper_1308_3214_amd import workloads as W
    n = 1024
    _, u0, _ = W.sine_modes_1d(n, seed=1)
    ms, _, info = run_plan((n,), 1.0 / (n - 1), 0, 1, 2.0, "f64", u0, steps, warmup, profile=False)
    return also_line(ms, steps, info, n)


def star_workload(steps=300, warmup=10, flags=0):
    """2048^2 star cavity, P = 3, CFL 1.5, FP32 (line objects, Sec. 4.3);
    flags = MOL_SYMMETRIC_D averages D over both sweep orders."""
    from paper_1308_3214_amd import workloads as W
    n = 2048
    dom, mask, cross = W.star_domain(n, seed=1)
    u0 = W.star_pulses(dom, mask, seed=1)
    ms, _, info = run_plan((n, n), 1.0 / (n - 1), 0, 3, 1.5, "f32", u0, steps, warmup,
                           profile=False, mask=mask, cross=cross, flags=flags)
    out = also_line(ms, steps, info, info["unknowns"])
    out["points"] = "inside nodes (%d)" % info["unknowns"]
    if not flags:
        u20 = solve_from_start((n, n), 1.0 / (n - 1), 0, 3, 1.5, "f32", u0, 20, mask=mask, cross=cross)
        out["error_u20"] = fixture_error("star2048_p3_cfl15_20", u20)
    return out


def closed_form_plane_waves(n, ks, ph, P, beta, alpha, nsteps):
    """Exact discrete solution of the 3D periodic scheme for plane-wave data
    (each wave an eigenvector: a scalar three-level recurrence with the
    symbols of C and D from the 40-digit symbol of L^{-1})."""
    import mpmath as mp
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import closed_forms as cf
    h = 1.0 / n
    x = np.arange(n) / n
    expect = np.zeros((n, n, n))
    for (kx, ky, kz), p in zip(ks, ph):
        Kg = [cf.khat(2 * mp.pi * int(k) * h, alpha * h) for k in (kx, ky, kz)]
        Dg = [1 - K for K in Kg]
        Ch = Kg[1] * Kg[2] * Dg[0] + Kg[2] * Kg[0] * Dg[1] + Kg[0] * Kg[1] * Dg[2]
        Dh = 1 - Kg[0] * Kg[1] * Kg[2]
        r = cf.rhs_symbol(P, beta, Ch, Dh)
        amp = float(cf.mode_sequence(r, 1, 1 + r / 2, nsteps)[nsteps])
        expect += 0.25 * amp * np.cos(2 * np.pi * (kx * x[None, None, :] + ky * x[None, :, None]
                                                   + kz * x[:, None, None]) + p)
    return expect


def periodic3d_workload(steps=200, warmup=10):
    """3D periodic 256^3, P = 2, CFL 2, FP32, four plane waves; error of u^200
    against the exact discrete solution."""
    import numpy as np
    from paper_1308_3214_amd import workloads as W
    n = 256
    u0, ks, ph = W.plane_waves_3d(n, seed=1)
    ms, _, info = run_plan((n, n, n), 1.0 / n, 1, 2, 2.0, "f32", u0, steps, warmup, profile=False)
    out = also_line(ms, steps, info, n ** 3)
    u200 = solve_from_start((n, n, n), 1.0 / n, 1, 2, 2.0, "f32", u0, 200)
    ex = closed_form_plane_waves(n, ks, ph, 2, info["beta"], info["alpha"], 200)
    out["error_u200"] = {"vs": "exact discrete solution (closed form, plane waves are eigenvectors)",
                         "rel_L2": float("%.3e" % (np.linalg.norm(u200 - ex) / np.linalg.norm(ex))),
                         "max_elem": float("%.3e" % (np.abs(u200 - ex).max() / np.abs(ex).max()))}
    return out


def source_workload(n=4096, steps=200, warmup=10):
    """The 4096^2 P = 2 FP32 CFL 2 step with a source term (mol_step_source):
    a Gaussian point source (width 3 h, centre of the square) times a
    sinusoid switched on smoothly, its fields at t_{n-1}, t_n, t_{n+1}
    resident in HBM; against plain mol_step on the same buffers (both
    eager, one launch per sweep)."""
    import numpy as np
    import torch
    from paper_1308_3214_amd import molt
    from paper_1308_3214_amd import workloads as W
    h = 1.0 / (n - 1)
    plan = molt.Plan((n, n), h, 0, P=2, cfl=2.0, dtype="f32")
    info = plan.info
    dt = 2.0 * h
    x = np.arange(n) * h - 0.5
    g = np.exp(-x ** 2 / (2 * (3 * h) ** 2))
    G = torch.tensor(np.outer(g, g) / (2 * np.pi * (3 * h) ** 2), dtype=torch.float32, device="cuda")
    w = 2 * np.pi / (40 * h)
    f = lambda t: np.sin(w * t) * (1 - np.exp(-(t / (200 * h)) ** 2))
    t0 = 100 * dt
    sp, sc, sn = G * f(t0 - dt), G * f(t0), G * f(t0 + dt)
    u = [torch.tensor(W.gaussian_pulses_2d(n, seed=1), dtype=torch.float32, device="cuda")
         for _ in range(3)]
    stream = torch.cuda.Stream()
    out = {}
    # the same source as f(t) G(x) through mol_solve_source: C[G] once, then
    # the fused steps with G and C[G] in their last launch
    CG = torch.empty_like(G)
    plan.apply("C", G, CG)
    fv = [f(t0 + (k - 1) * dt) for k in range(steps + 2)]
    with torch.cuda.stream(stream):
        plan.solve_source(u[0], u[1], warmup, G, CG, fv[:warmup + 2], stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.solve_source(u[0], u[1], steps, G, CG, fv, stream=stream)
        e1.record(stream)
        stream.synchronize()
    out["solve_source"] = e0.elapsed_time(e1) / steps
    for name, call in (("step_source", lambda a, b, c: plan.step_source(a, b, c, sp, sc, sn, stream=stream)),
                       ("step", lambda a, b, c: plan.step(a, b, c, stream=stream))):
        with torch.cuda.stream(stream):
            for k in range(warmup):
                call(u[k % 3], u[(k + 1) % 3], u[(k + 2) % 3])
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for k in range(steps):
                call(u[k % 3], u[(k + 1) % 3], u[(k + 2) % 3])
            e1.record(stream)
            stream.synchronize()
        out[name] = e0.elapsed_time(e1) / steps
    torch.cuda.synchronize()
    assert all(torch.isfinite(x).all().item() for x in u), "non-finite field"
    plan.close()
    ms = out["step_source"]
    return {"Mpoint-updates/s": round(n * n / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 5),
            "kernels": info["kernels_per_source_step"],
            "model_hbm_frac": round(info["bytes_per_source_step"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "plain_step_ms": round(out["step"], 5),
            "separable_source_solve_ms_per_step": round(out["solve_source"], 5)}


def fig3_workload(steps=20, reps=20):
    """The point-source run of the ADI section's figure: 81^2 nodes (80 x 80
    cells) on [-1, 1]^2, CFL 2, a discrete delta at the centre times a
    sinusoid switched on smoothly, FP64, P = 1 and 2, 20 steps (t = 1) through
    mol_solve_source from rest; wall time per step (a latency-bound size) and
    the field's largest value at t = 1."""
    import numpy as np
    import torch
    from paper_1308_3214_amd import molt
    from paper_1308_3214_amd import workloads as W
    G, f, h = W.point_source_fig3()
    out = []
    for P in (1, 2):
        plan = molt.Plan(G.shape, h, 0, P=P, cfl=2.0, dtype="f64")
        dt = plan.info["beta"] / plan.info["alpha"]
        fv = f(dt * np.arange(steps + 2))
        dG = torch.tensor(G, dtype=torch.float64, device="cuda")
        dCG = None
        if P == 2:
            dCG = torch.empty_like(dG)
            plan.apply("C", dG, dCG)
        A, B = torch.zeros_like(dG), torch.zeros_like(dG)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            plan.solve_source(A, B, steps, dG, dCG, fv, stream=stream)
            stream.synchronize()
            umax = float(B.abs().max())
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                A.zero_()
                B.zero_()
                plan.solve_source(A, B, steps, dG, dCG, fv, stream=stream)
            e1.record(stream)
            stream.synchronize()
        plan.close()
        out.append({"P": P, "steps": steps, "ms_per_step": round(e0.elapsed_time(e1) / (reps * steps), 5),
                    "max_abs_u_t1": round(umax, 6)})
    return out


# Table 3 of the paper (ADI refinement study, 641^2 on [-1, 1]^2, T = 1.2,
# dt = 0.025, beta = beta_max(P)): printed max-over-steps L2 error and run time
# in seconds; the paper states no hardware or precision.
PAPER_TABLE3_DT0025 = {1: (4.84e-3, 30.0), 2: (4.97e-5, 94.2), 3: (2.29e-6, 186.2)}


def table3_workload(P, dt=0.025, T=1.2, dtype="f64", reps=5):
    """The paper's ADI refinement workload on the GPU: sin(pi x) sin(pi y) on
    641^2 nodes, analytic u^1, steps to T; wall time of the whole run (graph
    replay, fields resident) and the max-over-steps L2 error against the exact
    standing mode (an untimed second pass)."""
    import numpy as np
    import torch
    from paper_1308_3214_amd import molt
    from paper_1308_3214_amd import workloads as W
    u0, h = W.table3_mode(641)
    om = np.sqrt(2.0) * np.pi
    nsteps = int(round(T / dt))
    plan = molt.Plan(u0.shape, h, 0, P=P, dt=dt, dtype=dtype)
    td = torch.float64 if dtype == "f64" else torch.float32
    a0 = torch.tensor(u0, dtype=td, device="cuda")
    b0 = torch.tensor(u0 * np.cos(om * dt), dtype=td, device="cuda")
    a, b = a0.clone(), b0.clone()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        plan.solve(a, b, nsteps - 1)            # warm: graph capture
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a.copy_(a0)
        b.copy_(b0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(st):
            e0.record(st)
            plan.solve(a, b, nsteps - 1)
            e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    # error pass: one step at a time
    ex = torch.tensor(u0, dtype=torch.float64, device="cuda")
    a.copy_(a0)
    b.copy_(b0)
    err = float(torch.sqrt(h * h * ((b.double() - ex * np.cos(om * dt)) ** 2).sum()))
    for s_ in range(2, nsteps + 1):
        plan.solve(a, b, 1)
        torch.cuda.synchronize()
        err = max(err, float(torch.sqrt(h * h * ((b.double() - ex * np.cos(om * s_ * dt)) ** 2).sum())))
    plan.close()
    run_ms = min(times)
    pe, pt = PAPER_TABLE3_DT0025.get(P, (None, None)) if abs(dt - 0.025) < 1e-12 else (None, None)
    return {"P": P, "dtype": dtype, "steps": nsteps, "run_ms": round(run_ms, 4),
            "ms_per_step": round(run_ms / (nsteps - 1), 5), "max_L2_error": float("%.3e" % err),
            "paper_max_L2_error": pe, "paper_run_s": pt}


def serve(count=256, rate_hz=50.0, seed=1, budget=2 << 30, nstreams=3, burst=False, steps=100,
          batched=False):
    """The serving workload: a Poisson stream of independent FP32 requests
    (n log-uniform in [128, 2048], P in {1, 2, 3}, CFL in [1, 4], 100 steps,
    4 Gaussian pulses) through the request server with a device budget.  Three
    compute streams and the server's copy stream fill the box's four hardware
    queues (a fifth stream would share a queue and wait behind its work).
    Latency = scheduled arrival -> completion seen by the polling loop; results
    are handed back in device memory.  batched: requests advance in rounds
    whose sweeps of one kernel run as one launch over all of them."""
    import numpy as np
    import torch
    from paper_1308_3214_amd import molt
    from paper_1308_3214_amd import workloads as W
    reqs = W.request_stream(count, rate_hz, seed, steps=steps, burst=burst)
    # initial fields in pinned host memory, made before the clock starts
    inits = [torch.from_numpy(W.request_initial(r).astype(np.float32)).pin_memory() for r in reqs]
    srv = molt.Server(budget, nstreams, batched=batched)
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
            r = reqs[rid_of[rid]]
            # the result handed to the client in device memory
            srv.result(rid, torch.empty((r.n, r.n), dtype=torch.float32, device="cuda"))
        if not got:
            time.sleep(50e-6)
        if tn > 300:
            raise RuntimeError("serving run did not finish")
    st = srv.stats()
    srv.close()
    lat = np.array([done_t[k] - arrival[k] for k in done_t]) * 1e3
    pts = float(sum(r.n * r.n * r.steps for r in reqs))
    span = max(done_t.values()) - min(r.arrival_s for r in reqs)
    out = {"requests": count, "rate_hz": None if burst else rate_hz, "burst": burst,
            "budget_bytes": budget, "mode": "batched rounds" if batched else "stream pool",
            "streams": 1 if batched else nstreams,
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3),
            "Mpoint-updates/s": round(pts / span / 1e6, 1),
            "span_s": round(span, 3), "peak_bytes": st["bytes_peak"],
            "admit_ms_mean": round(st["admit_seconds"] / count * 1e3, 3),
            "admit_ms_max": round(st["admit_max_seconds"] * 1e3, 3)}
    if batched:
        out.update(rounds=st["rounds"], launches=st["launches"], request_sweeps=st["sweeps"],
                   round_host_ms_mean=round(st["round_seconds"] / max(1, st["rounds"]) * 1e3, 4))
    return out


def plain_f64_vs_served(count=256, seed=1, steps=100, every=4):
    """The ordering target: the serving workload's requests solved one after
    another with plain FP64 plans (plan, start, graph-replayed solve, result in
    device memory, plan freed), against the same requests served in FP32
    (batched rounds, whole burst admitted).  Aggregate rates over the same
    point-updates; the served FP32 results compared with the FP64 ones on
    every `every`-th request (relative L2 per request)."""
    import numpy as np
    import torch
    from paper_1308_3214_amd import molt
    from paper_1308_3214_amd import workloads as W
    reqs = W.request_stream(count, 50.0, seed, steps=steps, burst=True)
    inits = [W.request_initial(r) for r in reqs]
    pts = float(sum(r.n * r.n * r.steps for r in reqs))
    ref = {}
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    gpu_ms = 0.0
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        plan = molt.Plan((r.n, r.n), 1.0 / (r.n - 1), 0, P=r.P, cfl=r.cfl, dtype="f64")
        a = torch.tensor(inits[i], dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            plan.start(a, b)
            plan.solve(a, b, r.steps - 1)
            e1.record(stream)
        stream.synchronize()
        gpu_ms += e0.elapsed_time(e1)
        if i % every == 0:
            ref[i] = b.cpu().numpy()
        plan.close()
    wall = time.perf_counter() - t0
    # the same requests served in FP32 (burst, batched rounds), results kept
    srv = molt.Server(32 << 30, 3, batched=True)
    rid_of = {}
    for i, r in enumerate(reqs):
        rid = srv.submit(inits[i], (r.n, r.n), 1.0 / (r.n - 1), r.steps, P=r.P, cfl=r.cfl, dtype="f32")
        rid_of[rid] = i
    errs = []
    left = set(rid_of)
    while left:
        for rid in srv.poll():
            i = rid_of[rid]
            got = srv.result(rid)
            left.discard(rid)
            if i in ref:
                errs.append(float(np.linalg.norm(got - ref[i]) / np.linalg.norm(ref[i])))
        time.sleep(1e-4)
    srv.close()
    return {"requests": count, "plain_f64_wall_s": round(wall, 3),
            "plain_f64_Mpoint-updates/s_wall": round(pts / wall / 1e6, 1),
            "plain_f64_gpu_s": round(gpu_ms * 1e-3, 3),
            "plain_f64_Mpoint-updates/s_gpu": round(pts / (gpu_ms * 1e-3) / 1e6, 1),
            "served_f32_vs_plain_f64_rel_L2_max": float("%.3e" % max(errs)),
            "served_f32_vs_plain_f64_rel_L2_median": float("%.3e" % float(np.median(errs))),
            "compared_requests": len(errs)}


def stream_copy(n_bytes=64 << 20, nsets=6, reps=24):
    """Measured device copy bandwidth, GB/s counting read + write: `nsets`
    buffer pairs rotated so that every copy starts from data outside the
    256 MB last-level cache (cold), and one pair copied repeatedly (warm)."""
    import torch
    src = [torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda") for _ in range(nsets)]
    dst = [torch.empty_like(x) for x in src]
    out = {}
    for name, k in (("cold", nsets), ("warm", 1)):
        for i in range(k):
            dst[i].copy_(src[i])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(reps):
            dst[i % k].copy_(src[i % k])
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(2.0 * n_bytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del src, dst
    return out


def cpu_baseline(n, P, cfl, nsteps=1, seed=1, reps=1, keep=None):
    """The FP64 oracle on the same workload: its start u^1, then `reps` timed
    windows of `nsteps` steps each (the median window gives the rate); `keep`
    (a list) receives the oracle's last field, u^(1 + reps * nsteps)."""
    import oracle
    from paper_1308_3214_amd import workloads as W
    h = 1.0 / (n - 1)
    b = oracle.beta_max(P)
    pb = oracle.Problem((n, n), h, oracle.DIRICHLET, b / (cfl * h))
    u0 = W.gaussian_pulses_2d(n, seed=seed)
    a, c = u0, pb.start(u0, P, b)
    times = []
    for _ in range(reps):
        t = time.perf_counter()
        a, c = pb.run(a, c, nsteps, P, b)
        times.append(time.perf_counter() - t)
    dt = sorted(times)[len(times) // 2]
    if keep is not None:
        keep.append(c)
    return {"value": n * n * nsteps / dt / 1e6, "unit": "Mpoint-updates/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "median of %d timed windows of %d step(s) of the %dx%d P=%d FP64 workload "
                      "(after the oracle's start): %s s" % (reps, nsteps, n, n, P,
                                                             ", ".join("%.2f" % x for x in times))}


def cpu_single_thread(n=1024, P=2, cfl=2.0, nsteps=2):
    """The same oracle on one thread (OMP_NUM_THREADS=1 in a child process, so
    this process keeps its thread pool), on a bounded sample."""
    import subprocess
    code = ("import json, bench; print(json.dumps(bench.cpu_baseline(%d, %d, %r, %d)))"
            % (n, P, cfl, nsteps))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError("single-thread oracle run failed: " + r.stderr[-2000:])
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--P", type=int, default=2)
    ap.add_argument("--cfl", type=float, default=2.0)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-also", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 64 MiB buffer 5 times (reference for the HBM byte counters)")
    ap.add_argument("--only", choices=["star", "periodic3d", "table3", "source", "fig3", "cfl"], default=None,
                    help="only run one secondary workload for --steps steps (for profiling)")
    args = ap.parse_args()
    if args.only == "table3":
        print(json.dumps({"table3": [table3_workload(P) for P in (1, 2, 3)]}))
        return
    if args.only == "fig3":
        print(json.dumps({"fig3": fig3_workload()}))
        return
    if args.only == "cfl":
        print(json.dumps({"cfl": cfl_lines(args.n, args.P, args.dtype, args.steps, args.warmup)}))
        return
    if args.only:
        fn = {"star": star_workload, "periodic3d": periodic3d_workload,
              "source": source_workload}[args.only]
        print(json.dumps({args.only: fn(steps=args.steps, warmup=args.warmup)}))
        return
    if args.copy_calibration:
        import torch
        src = torch.ones(16 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 64 << 20, "copies": 5}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver is built and measured on a single "
              "MI355X (multi-GPU slab decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    n, P = args.n, args.P
    # 15 calls: the first 3-6 calls after a plan is created run 3-7 % slower
    # than the rest (on fresh buffers, whatever the data), so the median of
    # 15 is the sustained rate of a long solve; every call is in rep_ms
    ms, kern, info = run_gpu(n, P, args.cfl, args.dtype, args.steps, args.warmup, reps=15)
    ms_step = ms / args.steps
    points = n * n
    value = points / (ms_step * 1e-3) / 1e6
    es = 8 if args.dtype == "f64" else 4
    # dominant kernel
    dom = max(range(len(kern)), key=lambda i: kern[i]["ms"])
    k = kern[dom]
    achieved = k["bytes"] / (k["ms"] * 1e-3) / 1e9
    tag = "%s_sweep_k%d" % (k["dir"], dom)
    traffic = traffic_for(tag)
    step_gbs = info["bytes_per_step"] / (ms_step * 1e-3) / 1e9
    ksum = sum(x["ms"] for x in kern)
    # the fixed model: 12 field passes per step for 2D P = 2 (every directional
    # sweep reads its input and writes its output once)
    model12 = 12 * es * points if (P == 2) else None
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
        "timing": {"reps": len(info["rep_ms"]), "steps_per_rep": args.steps, "rep_ms": info["rep_ms"],
                   "median_rep": True, "graphs_prepared": True,
                   "kernel_sum_ms_per_step": round(ksum, 5),
                   "ms_per_step_over_kernel_sum": round(ms_step / ksum, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": tag,
                     "kernel_ms": round(k["ms"], 5), "kernel_bytes": k["bytes"]},
        "step_bytes": info["bytes_per_step"],
        "stream_copy_GBs": stream_copy(),
        "step_hbm_frac": round(step_gbs / HBM_PEAK_GBS, 4),
        "step_hbm_frac_model12": (round(model12 / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                  if model12 else None),
        "kernels": [{"dir": x["dir"], "sweeps": x["sweeps"], "ms": round(x["ms"], 5),
                     "GB/s": round(x["bytes"] / (x["ms"] * 1e-3) / 1e9, 1)} for x in kern],
    }
    if n == 4096 and P == 2 and args.cfl == 2.0:
        from paper_1308_3214_amd import workloads as W
        u10 = solve_from_start((n, n), 1.0 / (n - 1), 0, P, args.cfl, args.dtype,
                               W.gaussian_pulses_2d(n, seed=1), 10)
        out["error_u10"] = fixture_error("adi4096_p2_cfl2_10", u10)
    if not args.no_also:
        also = {}
        import numpy as np
        from paper_1308_3214_amd import workloads as W
        fields = {}
        for dt in ("f64", "f32"):
            keep = []
            # both precisions run start + 10 + 3 x 500 steps: the FP32-vs-FP64
            # statement compares the same u^n
            ms2, _, inf2 = run_gpu(1024, 2, 2.0, dt, 500, 10, keep=keep)
            fields[dt] = keep[0]
            line = also_line(ms2, 500, inf2, 1024 * 1024)
            u500 = solve_from_start((1024, 1024), 1.0 / 1023, 0, 2, 2.0, dt,
                                    W.gaussian_pulses_2d(1024, seed=1), 500)
            line["error_u500"] = fixture_error("config2_1024_p2_cfl2_500", u500)
            also["1024x1024_P2_%s_500steps" % dt] = line
        also["1024x1024_P2_f32_vs_f64_rel_L2"] = float(
            "%.3e" % (np.linalg.norm(fields["f32"] - fields["f64"]) / np.linalg.norm(fields["f64"])))
        # the same workload with the two y sweeps of a step in separate launches
        # (v1 = C u written and read back): 11 field passes instead of 9
        from paper_1308_3214_amd import molt as _m
        ms2, kern2, inf2 = run_gpu(n, P, args.cfl, args.dtype, args.steps, args.warmup,
                                   flags=_m.SPLIT_Y)
        sp = also_line(ms2, args.steps, inf2, points)
        sp["kernels"] = [{"dir": x["dir"], "sweeps": x["sweeps"], "ms": round(x["ms"], 5),
                          "GB/s": round(x["bytes"] / (x["ms"] * 1e-3) / 1e9, 1)} for x in kern2]
        also["%dx%d_P%d_%s_split_y" % (n, n, P, args.dtype)] = sp
        k64 = max(20, args.steps // 4)
        ms2, kern64, inf2 = run_gpu(n, P, args.cfl, "f64", k64, 5)
        l64 = also_line(ms2, k64, inf2, points)
        l64["model12_hbm_frac"] = round(12 * 8 * points / (ms2 / k64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        l64["kernels"] = [{"dir": x["dir"], "sweeps": x["sweeps"], "ms": round(x["ms"], 5),
                           "GB/s": round(x["bytes"] / (x["ms"] * 1e-3) / 1e9, 1)} for x in kern64]
        if n == 4096 and P == 2 and args.cfl == 2.0:
            u10 = solve_from_start((n, n), 1.0 / (n - 1), 0, P, args.cfl, "f64",
                                   W.gaussian_pulses_2d(n, seed=1), 10)
            l64["error_u10"] = fixture_error("adi4096_p2_cfl2_10", u10)
        also["%dx%d_P%d_f64" % (n, n, P)] = l64
        also.update(cfl_lines(n, P, args.dtype, args.steps, args.warmup))
        also["line1d_1024_P1_f64_200steps"] = line1d_workload()
        also["paper_table3_641_dt0.025"] = [table3_workload(P) for P in (1, 2, 3)]
        also["star2048_P3_f32_300steps"] = star_workload()
        also["star2048_P3_f32_300steps_averaged_D"] = star_workload(flags=_m.SYMMETRIC_D)
        also["periodic3d_256_P2_f32_200steps"] = periodic3d_workload()
        also["source_4096_P2_f32_200steps"] = source_workload()
        also["paper_fig3_point_source_81x81_cfl2"] = fig3_workload()
        out["also"] = also
    if not args.no_serve:
        # stream pool (per-request graphs on three streams) and batched rounds
        # (one launch per kernel across all admitted requests)
        # admission-limited (2 GiB) and with the whole burst admitted (32 GiB)
        out["serving"] = {"poisson": serve(), "burst": serve(burst=True),
                          "batched": {"poisson": serve(batched=True),
                                      "burst": serve(burst=True, batched=True)},
                          "budget_32GiB": {"burst_pool": serve(burst=True, budget=32 << 30),
                                           "burst_batched": serve(burst=True, batched=True,
                                                                  budget=32 << 30)},
                          "plain_f64_sequential": plain_f64_vs_served()}
    if not args.no_cpu_baseline:
        import numpy as np
        from paper_1308_3214_amd import workloads as W
        keep = []
        out["cpu_baseline"] = cpu_baseline(n, P, args.cfl, 1, reps=3, keep=keep)
        out["cpu_baseline"]["single_thread"] = cpu_single_thread(1024, P, args.cfl, 2)
        # the headline's error against the oracle on the same seed and
        # workload: u^4 of the GPU (start and 3 steps) against the oracle's
        g4 = solve_from_start((n, n), 1.0 / (n - 1), 0, P, args.cfl, args.dtype,
                              W.gaussian_pulses_2d(n, seed=1), 4)
        r4 = keep[0]
        out["rel_L2_vs_oracle"] = float("%.3e" % (np.linalg.norm(g4 - r4) / np.linalg.norm(r4)))
        out["max_elem_vs_oracle"] = float("%.3e" % (np.abs(g4 - r4).max() / np.abs(r4).max()))
        out["vs_oracle_window"] = "u^4 (start + 3 steps), FP64 oracle, same seed and workload"
    print(json.dumps(out))


if __name__ == "__main__":
    main()
