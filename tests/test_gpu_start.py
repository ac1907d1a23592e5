"""GPU parity of the start with an initial velocity (mol_start with g; Sec.
3.2) against the oracle's start_g, and a started run of the Table 3 mode
against its 40-digit closed form.  g is scaled by 1 / dt so that the odd part
of u^1 is as large as the even part (tolerances as for every single step:
1e-12 FP64, 1e-5 FP32, relative L2 and per element)."""
import numpy as np
import pytest

import closed_forms as cf
from oracle import lines, scheme
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


CASES = [
    ((1000,), 1.0 / 999, 0, 2.0),
    ((129, 200), (1.0 / 199, 1.0 / 128), 0, 2.0),
    ((96, 257), 1.0 / 256, (0, 1), 1.5),
    ((20, 24, 28), 1.0 / 27, (0, 1, 0), 2.0),
    ("star", None, 0, 1.5),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("P", [1, 2, 3])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_start_with_velocity_parity(torch_cuda, molt, oracle_mod, case, P, dtype):
    torch = torch_cuda
    shape, h, bc, cfl = CASES[case]
    kw, okw, mask = {}, {}, None
    if shape == "star":
        dom, mask, cross = W.star_domain(120, seed=4)
        shape, h = mask.shape, 1.0 / 119
        kw = dict(mask=mask, cross=cross)
        okw = dict(segments=lines.segments(mask, cross), mask=mask)
    plan = molt.Plan(shape, h, bc, P=P, cfl=cfl, dtype=dtype, **kw)
    beta, alpha = plan.info["beta"], plan.info["alpha"]
    dt = beta / alpha
    # the 80-bit build of the oracle: on the star its FP64 build is itself
    # 1.5e-12 (per element) from the 80-bit one for this start, the GPU's FP64
    # result 1e-15 (the literal D = v - L^-1 v loses digits to cancellation)
    pb = oracle_mod.Problem(shape, h, bc, alpha, precision="ld", **okw)
    da = _dirichlet_axes(bc, len(shape))
    u0 = W.random_field(shape, seed=100 + case, dirichlet_axes=da)
    g = W.random_field(shape, seed=110 + case, dirichlet_axes=da) / dt
    if mask is not None:
        u0, g = u0 * mask, g * mask
    ref = pb.start_g(u0, g, P, beta)
    du0, dg = dev(torch, u0, dtype), dev(torch, g, dtype)
    out = torch.full_like(du0, float("nan"))
    plan.start(du0, out, g=dg)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    check("start with g %s P=%d" % (shape, P), got, ref, dtype)
    odd_ref = ref - pb.start(u0, P, beta)
    check("start with g %s P=%d, odd part" % (shape, P), got - pb.start(u0, P, beta), odd_ref, dtype)
    plan.close()


@pytest.mark.parametrize("P,dt", [(1, 0.05), (2, 0.05), (3, 0.1)])
def test_started_run_on_the_table3_grid(torch_cuda, molt, P, dt):
    # u = (cos(w t) + sin(w t)) sin(pi x) sin(pi y), w = sqrt(2) pi: u0 = phi,
    # g = w phi; u^1 from mol_start, then the graph-replayed solve, FP64
    torch = torch_cuda
    phi, h = W.table3_mode(641)
    w = np.sqrt(2.0) * np.pi
    plan = molt.Plan(phi.shape, h, 0, P=P, dt=dt, dtype="f64")
    ex = torch.tensor(phi, dtype=torch.float64, device="cuda")
    a = ex.clone()
    b = torch.empty_like(a)
    plan.start(a, b, g=ex * w)
    nsteps = int(round(1.2 / dt))
    err = float(torch.sqrt(h * h * ((b - ex * (np.cos(w * dt) + np.sin(w * dt))) ** 2).sum()))
    for s in range(2, nsteps + 1):
        plan.solve(a, b, 1)
        err = max(err, float(torch.sqrt(h * h * ((b - ex * (np.cos(w * s * dt) + np.sin(w * s * dt))) ** 2).sum())))
    torch.cuda.synchronize()
    plan.close()
    ref = float(cf.started_mode_error(P, dt, scheme.beta_max(P)))
    print("started run P=%d dt=%g: GPU max L2 error %.6e, closed form %.6e" % (P, dt, err, ref))
    assert abs(err / ref - 1) < 1e-8


def test_start_with_velocity_errors(torch_cuda, molt):
    torch = torch_cuda
    plan = molt.Plan((64, 64), 1.0 / 63, 0, P=2, cfl=2.0, dtype="f64")
    z = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    o = torch.zeros_like(z)
    with pytest.raises(molt.MolError):
        plan.start(z, o, g=o)                 # g overlaps u1
    plan.close()
