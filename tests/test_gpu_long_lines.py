"""x lines longer than one workgroup: chunks of 4096 nodes swept in two
passes with the carry table and scan of the exact strided sweeps between
them, exact across chunks (no truncation).

* 1D lines of 20 000 and 50 001 nodes (5 and 13 chunks, a ragged last
  chunk; 50 001 = 12 * 4096 + 1849), P = 1..3, FP64 and FP32: D_x, L^{-1}_x
  (taken as v - D v on chunked lines), rhs and a step against the FP64
  oracle; 9 steps of mol_solve against the oracle stepped 9 times (FP64).
* A last chunk of a single node (n = 3 * 4096 + 1): node M-1 lies in the
  previous chunk.
* 2D, 3 x 20 000 and 20 x 16 500 FP32 and FP64, P = 2: rhs and step
  (the fused solve programs need whole lines and fall back to the step).
* A line of 9 000 nodes, which fits one workgroup, swept both ways (the
  chunked configuration forced through the tuning interface): the same step
  to the FP64 bar.

The reference is the 80-bit build of the oracle: the FP64 build forms cell
widths from the coordinates j h, whose rounding grows with j (on a line of
50 001 nodes its D is 1.4e-12 from the 80-bit build, which agrees with an
independent numpy evaluation of the convolution to 1.7e-14).
"""
import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    return oracle


def _q(a, dtype):
    return np.asarray(a, np.float32).astype(np.float64) if dtype == "f32" else np.asarray(a)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [20000, 50001, 3 * 4096 + 1])
def test_long_1d_lines(torch_cuda, molt, oracle_mod, n, dtype):
    torch = torch_cuda
    h = 1.0 / (n - 1)
    g = np.random.default_rng(n)
    r = g.uniform(-1, 1, n)
    r[0] = r[-1] = 0.0
    r = _q(r, dtype)
    rd = dev(torch, r, dtype)
    out = torch.empty_like(rd)
    for P in (1, 2, 3):
        plan = molt.Plan((n,), h, 0, P=P, cfl=2.0, dtype=dtype)
        alpha, beta = plan.info["alpha"], plan.info["beta"]
        pb = oracle_mod.Problem((n,), h, 0, alpha, precision="ld")
        if P == 1:
            plan.apply("d_x", rd, out)
            torch.cuda.synchronize()
            check("long line n=%d D_x" % n, host(out), pb.Dg(r, 0), dtype)
            plan.apply("linv_x", rd, out)
            torch.cuda.synchronize()
            check("long line n=%d L^-1_x" % n, host(out), pb.linv(r, 0), dtype)
        plan.apply("rhs", rd, out)
        torch.cuda.synchronize()
        check("long line n=%d rhs P=%d" % (n, P), host(out), pb.rhs(r, P, beta), dtype)
        r2 = _q(g.uniform(-1, 1, n) * (np.arange(n) % (n - 1) != 0), dtype)
        a, b = dev(torch, r2, dtype), dev(torch, r, dtype)
        c = torch.empty_like(a)
        plan.step(a, b, c)
        torch.cuda.synchronize()
        check("long line n=%d step P=%d" % (n, P), host(c), pb.step(r2, r, P, beta), dtype)
        if dtype == "f64" and n == 50001:
            x = np.arange(n) * h
            u0 = np.sin(np.pi * x) + 0.3 * np.sin(5 * np.pi * x)
            u1 = pb.start(u0, P, beta)
            ra, rb = pb.run(u0, u1, 9, P, beta)
            a, b = dev(torch, u0, dtype), dev(torch, u1, dtype)
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                plan.solve(a, b, 9)
            torch.cuda.synchronize()
            check("long line n=%d solve 9 P=%d prev" % (n, P), host(a), ra, dtype)
            check("long line n=%d solve 9 P=%d curr" % (n, P), host(b), rb, dtype)
        plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(3, 20000), (20, 16500)])
def test_long_x_lines_2d(torch_cuda, molt, oracle_mod, shape, dtype):
    torch = torch_cuda
    ny, nx = shape
    h = (1.0 / (nx - 1), 1.0 / (ny - 1))
    plan = molt.Plan(shape, h, 0, P=2, cfl=2.0, dtype=dtype)
    alpha, beta = plan.info["alpha"], plan.info["beta"]
    pb = oracle_mod.Problem(shape, h, 0, alpha, precision="ld")
    r = _q(W.random_field(shape, seed=ny + nx, dirichlet_axes=(0, 1)), dtype)
    r2 = _q(W.random_field(shape, seed=ny + nx + 1, dirichlet_axes=(0, 1)), dtype)
    rd = dev(torch, r, dtype)
    out = torch.empty_like(rd)
    plan.apply("rhs", rd, out)
    torch.cuda.synchronize()
    check("long x lines %s rhs" % (shape,), host(out), pb.rhs(r, 2, beta), dtype)
    a = dev(torch, r2, dtype)
    plan.step(a, rd, out)
    torch.cuda.synchronize()
    check("long x lines %s step" % (shape,), host(out), pb.step(r2, r, 2, beta), dtype)
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_chunked_equals_whole_line(torch_cuda, molt, dtype):
    torch = torch_cuda
    n = 9000
    plan = molt.Plan((n,), 1.0 / (n - 1), 0, P=1, cfl=2.0, dtype=dtype)
    g = np.random.default_rng(9)
    up, uc = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    up[0] = up[-1] = uc[0] = uc[-1] = 0.0
    a, b = dev(torch, up, dtype), dev(torch, uc, dtype)
    whole, chunked = torch.empty_like(a), torch.empty_like(a)
    plan.step(a, b, whole)
    plan.set_kernel_config(0, 11)                     # the chunked configuration
    plan.step(a, b, chunked)
    torch.cuda.synchronize()
    check("n=9000 step chunked vs one workgroup", host(chunked), host(whole), dtype)
    plan.close()
