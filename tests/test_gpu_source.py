"""GPU parity of the step with a source term (mol_step_source) against the
FP64 oracle (Sec. 4, inclusion of source terms), and the forced-mode run on
the Table 3 grid against its closed form.

Tolerances: relative L2 1e-12 (FP64) and 1e-5 (FP32) for single steps on
seeded random fields (u zero on Dirichlet nodes, S nonzero everywhere); the
forced run reproduces the 40-digit closed form of the discrete scheme to
1e-8 relative in its max-over-steps error.
"""
import mpmath as mp
import numpy as np
import pytest

import closed_forms as cf
from oracle import scheme
from gpu_common import check, dev, rel
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


# (shape, h, bc, cfl): 1D, ragged 2D with several strided tiles, mixed and
# periodic boundaries, a 3D box
CASES = [
    ((1000,), 1.0 / 999, 0, 2.0),
    ((129, 200), (1.0 / 199, 1.0 / 128), 0, 2.0),
    ((96, 257), 1.0 / 256, (0, 1), 1.5),
    ((130, 70), 1.0 / 130, 1, 2.0),
    ((20, 24, 28), 1.0 / 27, (0, 1, 0), 2.0),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("P", [1, 2])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_step_source_parity(torch_cuda, molt, oracle_mod, case, P, dtype):
    torch = torch_cuda
    shape, h, bc, cfl = CASES[case]
    plan = molt.Plan(shape, h, bc, P=P, cfl=cfl, dtype=dtype)
    beta, alpha = plan.info["beta"], plan.info["alpha"]
    pb = oracle_mod.Problem(shape, h, bc, alpha)
    da = _dirichlet_axes(bc, len(shape))
    up = W.random_field(shape, seed=70 + case, dirichlet_axes=da)
    uc = W.random_field(shape, seed=80 + case, dirichlet_axes=da)
    # S of size 1 / (c dt)^2: the source part of the step is O(1), like rhs(u)
    a2 = (beta / alpha) ** 2
    s = [W.random_field(shape, seed=90 + 3 * case + k) / a2 for k in range(3)]
    ref = pb.step_source(up, uc, s[0], s[1], s[2], P, beta)
    t = [dev(torch, x, dtype) for x in (up, uc, *s)]
    out = torch.full_like(t[0], float("nan"))
    plan.step_source(t[0], t[1], out, t[2] if P == 2 else None, t[3], t[4] if P == 2 else None)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    check("source step %s P=%d" % (shape, P), got, ref, dtype)
    # the source part alone, so that a lost term of S is not hidden by rhs(u)
    check("source step %s P=%d, source part" % (shape, P), got - pb.step(up, uc, P, beta),
          ref - pb.step(up, uc, P, beta), dtype)
    # u_next may alias u_prev, as for mol_step
    plan.step_source(t[0], t[1], t[0], t[2] if P == 2 else None, t[3], t[4] if P == 2 else None)
    torch.cuda.synchronize()
    check("source step in place %s P=%d" % (shape, P), t[0].double().cpu().numpy(), ref, dtype)
    plan.close()


@pytest.mark.parametrize("P,dt", [(1, 0.05), (2, 0.05), (2, 0.025)])
def test_forced_mode_on_the_table3_grid(torch_cuda, molt, P, dt):
    # u_tt = laplacian(u) + S on [-1, 1]^2, S = (2 pi^2 - 4) cos(2t) phi, exact
    # u = cos(2t) phi; 641^2 nodes, T = 1.2, FP64
    torch = torch_cuda
    phi, h = W.table3_mode(641)
    w0 = 2.0
    nsteps = int(round(1.2 / dt))
    plan = molt.Plan(phi.shape, h, 0, P=P, dt=dt, dtype="f64")
    beta = plan.info["beta"]
    assert abs(beta - scheme.beta_max(P)) < 1e-12
    ph = torch.tensor(phi, dtype=torch.float64, device="cuda")
    g = lambda t: (2 * np.pi ** 2 - w0 ** 2) * np.cos(w0 * t)
    a, b = ph.clone(), ph * np.cos(w0 * dt)
    c = torch.empty_like(ph)
    err = 0.0
    for k in range(1, nsteps):
        t = k * dt
        sp, sc, sn = ph * g(t - dt), ph * g(t), ph * g(t + dt)
        plan.step_source(a, b, c, sp if P == 2 else None, sc, sn if P == 2 else None)
        a, b, c = b, c, a
        err = max(err, float(torch.sqrt(h * h * ((b - ph * np.cos(w0 * (k + 1) * dt)) ** 2).sum())))
    torch.cuda.synchronize()
    plan.close()
    ref = float(cf.forced_mode_error(P, dt, scheme.beta_max(P)))
    print("forced mode P=%d dt=%g: GPU max L2 error %.6e, closed form %.6e" % (P, dt, err, ref))
    assert abs(err / ref - 1) < 1e-8, (P, dt, err, ref)


def test_step_source_errors(torch_cuda, molt):
    torch = torch_cuda
    shape = (64, 64)
    z = torch.zeros(shape, dtype=torch.float64, device="cuda")
    o = torch.zeros_like(z)
    p3 = molt.Plan(shape, 1.0 / 63, 0, P=3, cfl=2.0, dtype="f64")
    with pytest.raises(molt.MolError) as ei:
        p3.step_source(z, z, o, z, z, z)
    assert ei.value.status == molt.MOL_E_UNSUPPORTED
    p3.close()
    p2 = molt.Plan(shape, 1.0 / 63, 0, P=2, cfl=2.0, dtype="f64")
    with pytest.raises(molt.MolError):
        p2.step_source(z, z, o, None, z, None)          # P = 2 needs three levels
    s = torch.zeros_like(z)
    with pytest.raises(molt.MolError):
        p2.step_source(z, z, s, z, s, z)                # u_next overlaps s_curr
    p2.close()
