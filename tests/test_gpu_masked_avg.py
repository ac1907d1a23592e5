"""GPU parity of masked plans with MOL_SYMMETRIC_D (D averaged over both
orders of the directional inverses; Sec. 4, operation count) against the
oracle's D_avg and Table 2 schedule, and the property the averaging buys: on
the ellipse of the ADI section (symmetric under x <-> y) a run from the
transposed data is the transpose of the run, which the literal D does not give.
"""
import numpy as np
import pytest

from oracle import lines
from gpu_common import TOL, check, dev, host
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


def domain(kind):
    if kind == "ellipse":
        mask, cross = W.ellipse_domain(80)
        return mask, cross, 1.0 / 79, 2.0
    dom, mask, cross = W.star_domain(120, seed=2)
    return mask, cross, 1.0 / 119, 1.5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["ellipse", "star"])
def test_averaged_d_operators_and_steps(torch_cuda, molt, oracle_mod, kind, dtype):
    torch = torch_cuda
    mask, cross, h, cfl = domain(kind)
    shape = mask.shape
    segs = lines.segments(mask, cross)
    v = W.random_field(shape, seed=17) * mask
    w = W.random_field(shape, seed=18) * mask
    vd, wd = dev(torch, v, dtype), dev(torch, w, dtype)
    out = torch.empty_like(vd)
    for P in (2, 3):
        plan = molt.Plan(shape, h, 0, P=P, cfl=cfl, dtype=dtype, mask=mask, cross=cross,
                         flags=molt.SYMMETRIC_D)
        beta = plan.info["beta"]
        pb = oracle_mod.Problem(shape, h, 0, plan.info["alpha"], segments=segs, mask=mask)
        if P == 2:
            plan.apply("D", vd, out)
            torch.cuda.synchronize()
            check("%s averaged D" % kind, host(out), pb.D_avg(v), dtype)
            plan.apply("C", vd, out)
            torch.cuda.synchronize()
            check("%s C" % kind, host(out), pb.C(v), dtype)
        plan.apply("rhs", vd, out)
        torch.cuda.synchronize()
        check("%s rhs P=%d" % (kind, P), host(out), pb.rhs_with(v, P, beta, pb.D_avg), dtype)
        plan.step(wd, vd, out)
        torch.cuda.synchronize()
        check("%s step P=%d" % (kind, P), host(out), pb.step_avg(w, v, P, beta), dtype)
        # 9 steps on a non-default stream (one captured 8-step graph and one
        # step launched directly) against the oracle stepped as often, from
        # smooth data (a Gaussian of width 0.15 at the centre): random data
        # put single FP32 nodes next to short end cells at 1.2e-5 of max |u|
        # in some steps (rel L2 2e-6), rounding of the end-cell forcing
        ny, nx = shape
        yy, xx = np.meshgrid(np.arange(ny) / (ny - 1), np.arange(nx) / (nx - 1), indexing="ij")
        gs = np.exp(-((xx - 0.5) ** 2 + (yy - 0.5) ** 2) / (2 * 0.15 ** 2)) * mask
        vs, ws = gs, gs * 0.9
        a, b = dev(torch, ws, dtype), dev(torch, vs, dtype)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            plan.solve(a, b, 9)
        torch.cuda.synchronize()
        ra, rb = ws, vs
        for _ in range(9):
            ra, rb = rb, pb.step_avg(ra, rb, P, beta)
        check("%s solve 9 P=%d prev" % (kind, P), host(a), ra, dtype)
        check("%s solve 9 P=%d" % (kind, P), host(b), rb, dtype)
        plan.close()


def test_averaged_d_run_commutes_with_transposition(torch_cuda, molt):
    torch = torch_cuda
    mask, cross, h, cfl = domain("ellipse")
    assert np.array_equal(mask, mask.T)
    u0 = W.random_field(mask.shape, seed=19) * mask
    res = {}
    for name, flags in (("averaged", molt.SYMMETRIC_D), ("literal", 0)):
        plan = molt.Plan(mask.shape, h, 0, P=2, cfl=cfl, dtype="f64", mask=mask, cross=cross,
                         flags=flags)
        runs = []
        for x in (u0, np.ascontiguousarray(u0.T)):
            a = dev(torch, x, "f64")
            b = torch.empty_like(a)
            plan.start(a, b)
            plan.solve(a, b, 20)
            torch.cuda.synchronize()
            runs.append(host(b))
        plan.close()
        res[name] = np.linalg.norm(runs[1] - runs[0].T) / np.linalg.norm(runs[0])
        print("%s D: 20 steps from u0 and from u0^T, transposition defect %.3e" % (name, res[name]))
    assert res["averaged"] < 1e-12
    assert res["literal"] > 1e-6
