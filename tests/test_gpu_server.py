"""GPU tests of the request server (serving many independent solves), in both
modes (stream pool; batched rounds whose launches carry many requests): every
result of a mixed, queued workload equals the same request solved alone
(bitwise: the same kernels on the same data), one small request matches the
80-bit oracle, admission respects the device budget, and failures are
reported per request."""
import numpy as np
import pytest

from oracle import lines
from paper_1308_3214_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def molt(torch_cuda):
    from paper_1308_3214_amd import molt as m
    return m


def _alone(torch, molt, u0, shape, h, nsteps, **kw):
    plan = molt.Plan(shape, h, 0, **kw)
    dt = torch.float64 if kw.get("dtype", "f64") == "f64" else torch.float32
    a = torch.tensor(u0, dtype=dt, device="cuda")
    b = torch.empty_like(a)
    plan.start(a, b)
    if nsteps > 1:
        plan.solve(a, b, nsteps - 1)
    torch.cuda.synchronize()
    plan.close()
    return b.cpu().numpy()


def _mix():
    dom, mask, cross = W.star_domain(150, seed=4)
    reqs = []
    rng = np.random.default_rng(5)
    for i, (n, P, dt) in enumerate([(100, 1, "f32"), (257, 2, "f32"), (600, 3, "f32"),
                                    (130, 2, "f64"), (300, 3, "f64"), (420, 1, "f32"),
                                    (77, 3, "f32"), (513, 2, "f64"), (257, 2, "f32")]):
        cfl = float(rng.uniform(1.0, 4.0))
        u0 = W.gaussian_pulses_2d(n, seed=30 + i, npulses=4)
        reqs.append(dict(u0=u0, shape=(n, n), h=1.0 / (n - 1), nsteps=5 + i,
                         kw=dict(P=P, cfl=cfl, dtype=dt)))
    u0 = W.star_pulses(dom, mask, seed=4, npulses=3, sigma=0.05)
    reqs.append(dict(u0=u0, shape=mask.shape, h=1.0 / 149, nsteps=9,
                     kw=dict(P=3, cfl=1.5, dtype="f32", mask=mask, cross=cross)))
    return reqs


@pytest.mark.parametrize("batched", [False, True])
def test_mixed_requests_equal_alone(torch_cuda, molt, batched):
    torch = torch_cuda
    reqs = _mix()
    # a budget that holds only a few requests at a time: admission queues
    def foot(r):
        es = 8 if r["kw"]["dtype"] == "f64" else 4
        return (molt.workspace_bytes(shape=r["shape"], h=r["h"], **r["kw"])
                + 2 * es * int(np.prod(r["shape"])))
    budget = int(1.1 * max(foot(r) for r in reqs))
    assert sum(foot(r) for r in reqs) > 1.4 * budget      # admission must queue
    srv = molt.Server(budget, nstreams=4, batched=batched)
    ids = [srv.submit(r["u0"], r["shape"], r["h"], r["nsteps"], **r["kw"]) for r in reqs]
    done = set()
    import time
    t0 = time.time()
    while len(done) < len(ids):
        done.update(srv.poll())
        assert time.time() - t0 < 60, "server did not finish"
        time.sleep(0.001)
    st = srv.stats()
    assert st["bytes_peak"] <= budget and st["completed"] == len(ids)
    if batched:
        # some launches carried the sweeps of several requests
        print("rounds", st["rounds"], "launches", st["launches"], "request sweeps", st["sweeps"])
        assert st["rounds"] > 0 and st["sweeps"] > st["launches"]
    for rid, r in zip(ids, reqs):
        got = srv.result(rid)
        # the batched server's plans take the size-independent configurations
        kw = dict(r["kw"], flags=molt.UNIFORM_CONFIG) if batched else r["kw"]
        ref = _alone(torch, molt, r["u0"], r["shape"], r["h"], r["nsteps"], **kw)
        print("request", rid, r["shape"], r["kw"].get("P"), r["kw"].get("dtype"),
              "max |mix - alone| =", float(np.abs(got - ref).max()))
        assert np.array_equal(got, ref), rid
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()


@pytest.mark.parametrize("batched", [False, True])
def test_server_result_matches_oracle(torch_cuda, molt, oracle_mod, batched):
    n, P, nsteps = 96, 2, 8
    h = 1.0 / (n - 1)
    u0 = W.gaussian_pulses_2d(n, seed=8, npulses=3, sigma=0.05)
    srv = molt.Server(1 << 30, nstreams=2, batched=batched)
    rid = srv.submit(u0, (n, n), h, nsteps, P=P, cfl=2.0, dtype="f64")
    import time
    t0 = time.time()
    while rid not in srv.poll():
        assert time.time() - t0 < 30
        time.sleep(0.001)
    got = srv.result(rid)
    beta = molt.beta_max(P)
    pb = oracle_mod.Problem((n, n), h, 0, beta / (2.0 * h), precision="ld")
    _, ref = pb.run(u0, pb.start(u0, P, beta), nsteps - 1, P, beta)
    e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("server vs 80-bit oracle rel L2 =", e)
    assert e < 1e-12
    srv.close()


@pytest.mark.parametrize("batched", [False, True])
def test_server_budget_and_errors(torch_cuda, molt, batched):
    srv = molt.Server(1 << 20, nstreams=1, batched=batched)
    u0 = np.zeros((512, 512))
    with pytest.raises(molt.MolError):
        srv.submit(u0, (512, 512), 1 / 511, 3, P=2, cfl=2.0, dtype="f64")     # > budget
    with pytest.raises(molt.MolError):
        srv.submit(np.zeros((8, 8)), (8, 8), 1 / 7, 3, P=9, cfl=2.0)           # invalid P
    assert srv.stats()["queued"] == 0
    srv.close()


def test_batched_serving_stream_equals_alone(torch_cuda, molt):
    # a burst of requests drawn like the serving workload (smaller sides and
    # fewer steps): in batched rounds, each result is bitwise the solve alone
    torch = torch_cuda
    reqs = W.request_stream(24, 50.0, seed=3, steps=12, nmax=512, burst=True)
    srv = molt.Server(1 << 30, nstreams=1, batched=True)
    ids = []
    for r in reqs:
        n = r.n
        u0 = W.request_initial(r).astype(np.float32)
        ids.append((srv.submit(u0, (n, n), 1.0 / (n - 1), r.steps, P=r.P, cfl=r.cfl, dtype="f32"),
                    u0, n, r))
    done = set()
    import time
    t0 = time.time()
    while len(done) < len(ids):
        done.update(srv.poll())
        assert time.time() - t0 < 60, "server did not finish"
        time.sleep(0.001)
    st = srv.stats()
    print("rounds", st["rounds"], "launches", st["launches"], "request sweeps", st["sweeps"])
    assert st["sweeps"] > st["launches"]
    for rid, u0, n, r in ids:
        got = srv.result(rid)
        ref = _alone(torch, molt, u0, (n, n), 1.0 / (n - 1), r.steps, P=r.P, cfl=r.cfl, dtype="f32",
                     flags=molt.UNIFORM_CONFIG)
        assert np.array_equal(got, ref), (rid, n, r.P)
    srv.close()
