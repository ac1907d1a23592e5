"""The benchmark workloads at their full sizes, in the launch configuration
the benchmark times (mol_solve from mol_start, tuned kernels), checked against
what the oracle can compute at that size or against exact properties:

* 3D periodic 256^3, P = 2, CFL 2, 200 steps: four plane waves are
  eigenvectors of the discrete scheme, so the exact discrete solution is a
  scalar recurrence per wave (symbols by 40-digit quadrature, closed_forms).
* 2D 4096^2 Dirichlet, P = 2, CFL 2: start + 2 steps against the FP64 oracle.
* 2D 1024^2 Dirichlet, P = 2, FP64, 500 steps: the leapfrog energy
  |u^{n+1} - u^n|^2 + <u^{n+1}, K u^n> (K = -rhs, symmetric on a rectangle)
  is conserved by the scheme; the GPU operator keeps it to rounding.
* 2D 2048^2 star cavity, P = 3, CFL 1.5: one step against the FP64 oracle on
  the line objects, and 300 steps stay bounded and zero outside.
"""
import mpmath as mp
import numpy as np
import pytest

import closed_forms as cf
from oracle import lines, scheme
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_3d_periodic_256_plane_waves(torch_cuda, molt, dtype):
    torch = torch_cuda
    n, P, cfl, nsteps = 256, 2, 2.0, 200
    h = 1.0 / n
    u0, ks, ph = W.plane_waves_3d(n, seed=1)
    plan = molt.Plan((n, n, n), h, 1, P=P, cfl=cfl, dtype=dtype)
    beta, alpha = plan.info["beta"], plan.info["alpha"]
    td = torch.float64 if dtype == "f64" else torch.float32
    a = torch.tensor(u0, dtype=td, device="cuda")
    b = torch.empty_like(a)
    plan.start(a, b)
    plan.solve(a, b, nsteps - 1)
    torch.cuda.synchronize()
    got = b.double().cpu().numpy()
    x = np.arange(n) / n
    expect = np.zeros_like(u0)
    for (kx, ky, kz), p in zip(ks, ph):
        Kg = [cf.khat(2 * mp.pi * int(k) * h, alpha * h) for k in (kx, ky, kz)]
        Dg = [1 - K for K in Kg]
        Ch = Kg[1] * Kg[2] * Dg[0] + Kg[2] * Kg[0] * Dg[1] + Kg[0] * Kg[1] * Dg[2]
        Dh = 1 - Kg[0] * Kg[1] * Kg[2]
        r = cf.rhs_symbol(P, beta, Ch, Dh)
        amp = float(cf.mode_sequence(r, 1, 1 + r / 2, nsteps)[nsteps])
        expect += 0.25 * amp * np.cos(2 * np.pi * (kx * x[None, None, :] + ky * x[None, :, None]
                                                   + kz * x[:, None, None]) + p)
    e = rel(got, expect)
    print("3D 256^3 %s 200 steps vs closed form: rel L2 = %.3e" % (dtype, e))
    # FP64: rounding level; FP32: 200 steps of single-precision sweeps
    assert e < (1e-11 if dtype == "f64" else 5e-5), e
    plan.close()


def test_2d_4096_steps_vs_oracle(torch_cuda, molt, oracle_mod):
    torch = torch_cuda
    n, P, cfl = 4096, 2, 2.0
    h = 1.0 / (n - 1)
    u0 = W.gaussian_pulses_2d(n, seed=1)
    plan = molt.Plan((n, n), h, 0, P=P, cfl=cfl, dtype="f32")
    beta = plan.info["beta"]
    a = torch.tensor(u0, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    plan.start(a, b)
    plan.solve(a, b, 2)
    torch.cuda.synchronize()
    pb = oracle_mod.Problem((n, n), h, 0, plan.info["alpha"])
    _, ref = pb.run(u0, pb.start(u0, P, beta), 2, P, beta)
    e = rel(b.double().cpu().numpy(), ref)
    print("4096^2 f32 start + 2 steps vs FP64 oracle: rel L2 = %.3e" % e)
    assert e < 1e-5
    plan.close()


def test_2d_1024_f64_500_steps_energy(torch_cuda, molt):
    torch = torch_cuda
    n, P, cfl, nsteps = 1024, 2, 2.0, 500
    h = 1.0 / (n - 1)
    u0 = W.gaussian_pulses_2d(n, seed=1)
    plan = molt.Plan((n, n), h, 0, P=P, cfl=cfl, dtype="f64")
    a = torch.tensor(u0, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    r = torch.empty_like(a)
    plan.start(a, b)

    def energy(x, y):
        plan.apply("rhs", x, r)
        return float(((y - x) ** 2).sum() - (y * r).sum())
    E0 = energy(a, b)
    plan.solve(a, b, nsteps - 1)
    E1 = energy(a, b)
    torch.cuda.synchronize()
    mx = float(b.abs().max())
    print("1024^2 f64 500 steps: energy %.15e -> %.15e (rel %.2e), max |u| %.3f"
          % (E0, E1, abs(E1 - E0) / abs(E0), mx))
    assert abs(E1 - E0) < 1e-10 * abs(E0)
    assert mx < 2 * float(np.abs(u0).max())
    plan.close()


def test_2d_2048_star_p3(torch_cuda, molt, oracle_mod):
    torch = torch_cuda
    n, P, cfl = 2048, 3, 1.5
    h = 1.0 / (n - 1)
    dom, mask, cross = W.star_domain(n, seed=1)
    u0 = W.star_pulses(dom, mask, seed=1)
    plan = molt.Plan((n, n), h, 0, P=P, cfl=cfl, dtype="f32", mask=mask, cross=cross)
    beta = plan.info["beta"]
    segs = lines.segments(mask, cross)
    pb = oracle_mod.Problem((n, n), h, 0, plan.info["alpha"], segments=segs, mask=mask)
    u1 = pb.start(u0, P, beta)
    a = torch.tensor(u0, dtype=torch.float32, device="cuda")
    b = torch.tensor(u1, dtype=torch.float32, device="cuda")
    o = torch.empty_like(a)
    plan.step(a, b, o)
    torch.cuda.synchronize()
    e = rel(o.double().cpu().numpy(), pb.step(u0, u1, P, beta))
    print("2048^2 star P=3 f32 step vs FP64 oracle: rel L2 = %.3e" % e)
    assert e < 1e-5
    plan.start(a, b)
    plan.solve(a, b, 299)
    torch.cuda.synchronize()
    got = b.cpu().numpy()
    assert np.isfinite(got).all() and np.abs(got).max() < 2 * np.abs(u0).max()
    assert (got[mask == 0] == 0).all()
    plan.close()
