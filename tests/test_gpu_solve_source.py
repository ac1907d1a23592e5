"""GPU parity of mol_solve_source (separable source S = f(t) G(x), Sec. 4,
inclusion of source terms) against the oracle's step with S^m = f_m G, and
the forced mode of the Table 3 grid against its closed form.  In 2D with
P = 2 the steps are mol_solve's fused ones (the chained walk in FP32), so
this also checks that G and C[G] reach the last launch with the right weights
every step."""
import numpy as np
import pytest

import closed_forms as cf
from oracle import scheme
from gpu_common import check, dev
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


def _dirichlet_axes(bc, nd):
    bb = list(bc) if np.ndim(bc) else [bc] * nd
    return tuple(a for a in range(nd) if bb[a] == 0)


# (shape, h, bc, cfl, P, dtype, nsteps, split_y)
CASES = [
    ((300, 260), 1.0 / 299, 0, 2.0, 2, "f32", 5, False),       # fused, chained walk
    ((300, 260), 1.0 / 299, 0, 2.0, 2, "f64", 4, False),       # fused, split y sweeps
    ((300, 260), 1.0 / 299, 0, 2.0, 2, "f32", 5, True),        # FP32 fused without the walk
    ((96, 257), 1.0 / 256, (0, 1), 1.5, 2, "f32", 4, False),
    ((129, 200), (1.0 / 199, 1.0 / 128), 0, 2.0, 1, "f64", 5, False),
    ((1000,), 1.0 / 999, 0, 2.0, 2, "f64", 5, False),
    ((20, 24, 28), 1.0 / 27, (0, 1, 0), 2.0, 2, "f32", 3, False),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_solve_source_parity(torch_cuda, molt, oracle_mod, case):
    torch = torch_cuda
    shape, h, bc, cfl, P, dtype, nsteps, split = CASES[case]
    plan = molt.Plan(shape, h, bc, P=P, cfl=cfl, dtype=dtype, flags=molt.SPLIT_Y if split else 0)
    if case == 0:
        assert plan.info["kernels_per_step"] == 2      # the chained fused step
    if split:
        assert plan.info["kernels_per_step"] == 3
    beta, alpha = plan.info["beta"], plan.info["alpha"]
    a2 = (beta / alpha) ** 2
    pb = oracle_mod.Problem(shape, h, bc, alpha)
    da = _dirichlet_axes(bc, len(shape))
    u0 = W.random_field(shape, seed=130 + case, dirichlet_axes=da)
    u1 = W.random_field(shape, seed=140 + case, dirichlet_axes=da)
    G = W.random_field(shape, seed=150 + case) / a2          # source part O(1)
    f = np.cos(0.7 * np.arange(nsteps + 2)) + 0.3
    a, b = u0, u1
    for k in range(nsteps):
        a, b = b, pb.step_source(a, b, f[k] * G, f[k + 1] * G, f[k + 2] * G, P, beta)
    dA, dB, dG = dev(torch, u0, dtype), dev(torch, u1, dtype), dev(torch, G, dtype)
    dCG = None
    if P == 2:
        dCG = torch.empty_like(dG)
        plan.apply("C", dG, dCG)
    plan.solve_source(dA, dB, nsteps, dG, dCG, f)
    torch.cuda.synchronize()
    for name, got, ref in (("prev", dA, a), ("curr", dB, b)):
        check("solve_source %s P=%d %d steps %s" % (shape, P, nsteps, name),
              got.double().cpu().numpy(), ref, dtype)
    plan.close()


@pytest.mark.parametrize("P,dt", [(1, 0.05), (2, 0.05)])
def test_solve_source_forced_mode(torch_cuda, molt, P, dt):
    # u_tt = laplacian(u) + g(t) phi on [-1, 1]^2, exact u = cos(2t) phi; 641^2
    # nodes, FP64, one step per call to record the max over steps
    torch = torch_cuda
    phi, h = W.table3_mode(641)
    w0 = 2.0
    nsteps = int(round(1.2 / dt))
    plan = molt.Plan(phi.shape, h, 0, P=P, dt=dt, dtype="f64")
    ph = torch.tensor(phi, dtype=torch.float64, device="cuda")
    CG = None
    if P == 2:
        CG = torch.empty_like(ph)
        plan.apply("C", ph, CG)
    g = lambda t: (2 * np.pi ** 2 - w0 ** 2) * np.cos(w0 * t)
    a, b = ph.clone(), ph * np.cos(w0 * dt)
    err = 0.0
    for k in range(1, nsteps):
        plan.solve_source(a, b, 1, ph, CG, [g((k - 1) * dt), g(k * dt), g((k + 1) * dt)])
        err = max(err, float(torch.sqrt(h * h * ((b - ph * np.cos(w0 * (k + 1) * dt)) ** 2).sum())))
    torch.cuda.synchronize()
    plan.close()
    ref = float(cf.forced_mode_error(P, dt, scheme.beta_max(P)))
    print("solve_source forced mode P=%d dt=%g: GPU %.6e, closed form %.6e" % (P, dt, err, ref))
    assert abs(err / ref - 1) < 1e-8


def test_solve_source_errors(torch_cuda, molt):
    torch = torch_cuda
    z = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    A, B, G = z.clone(), z.clone(), z.clone()
    p = molt.Plan((64, 64), 1.0 / 63, 0, P=2, cfl=2.0, dtype="f64")
    with pytest.raises(molt.MolError):
        p.solve_source(A, B, 2, G, None, [0.0] * 4)          # P = 2 needs C[G]
    with pytest.raises(ValueError):
        p.solve_source(A, B, 2, G, G, [0.0] * 3)             # nsteps + 2 values
    p.close()
    p = molt.Plan((64, 64), 1.0 / 63, 0, P=2, cfl=2.0, dtype="f64", flags=molt.INCREMENT_FORM)
    with pytest.raises(molt.MolError) as ei:
        p.solve_source(A, B, 2, G, G, [0.0] * 4)
    assert ei.value.status == molt.MOL_E_UNSUPPORTED
    p.close()
    mask = np.zeros((40, 40), np.uint8)
    mask[1:-1, 1:-1] = 1
    p = molt.Plan((40, 40), 1.0 / 39, 0, P=2, cfl=2.0, dtype="f64", mask=mask)
    z2 = torch.zeros((40, 40), dtype=torch.float64, device="cuda")
    with pytest.raises(molt.MolError) as ei:
        p.solve_source(z2.clone(), z2.clone(), 1, z2, z2, [0.0] * 3)
    assert ei.value.status == molt.MOL_E_UNSUPPORTED
    with pytest.raises(molt.MolError) as ei:
        p.step_source(z2, z2.clone(), z2.clone(), z2, z2, z2)
    assert ei.value.status == molt.MOL_E_UNSUPPORTED
    p.close()


@pytest.mark.parametrize("P", [1, 2])
def test_point_source_run_of_the_figure(torch_cuda, molt, oracle_mod, P):
    # 81^2 nodes on [-1, 1]^2, CFL 2, discrete delta at the centre switched on
    # smoothly; u^0 = u^1 = 0 (f and its derivatives vanish at t = 0); 20
    # steps (t = 1) through mol_solve_source against the oracle, FP64
    torch = torch_cuda
    G, f, h = W.point_source_fig3()
    plan = molt.Plan(G.shape, h, 0, P=P, cfl=2.0, dtype="f64")
    beta, alpha = plan.info["beta"], plan.info["alpha"]
    dt = beta / alpha
    nsteps = 20
    fv = f(dt * np.arange(nsteps + 2))               # f(t_0) .. f(t_{nsteps+1})
    pb = oracle_mod.Problem(G.shape, h, 0, alpha)
    a, b = np.zeros_like(G), np.zeros_like(G)
    for k in range(nsteps):
        a, b = b, pb.step_source(a, b, fv[k] * G, fv[k + 1] * G, fv[k + 2] * G, P, beta)
    dG = dev(torch, G, "f64")
    dCG = None
    if P == 2:
        dCG = torch.empty_like(dG)
        plan.apply("C", dG, dCG)
    A, B = torch.zeros_like(dG), torch.zeros_like(dG)
    plan.solve_source(A, B, nsteps, dG, dCG, fv)
    torch.cuda.synchronize()
    got = B.double().cpu().numpy()
    print("figure point source P=%d, 20 steps: max|u| %.3e" % (P, np.abs(b).max()))
    assert np.abs(b).max() > 1e-3
    check("figure point source P=%d, 20 steps" % P, got, b, "f64")
    plan.close()
