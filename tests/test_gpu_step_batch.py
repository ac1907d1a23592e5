"""mol_step_batch through the C-ABI: one step of many independent plans with
the launches that share a kernel instantiation batched into one launch.

The results must be those of mol_step on each plan, bit for bit (the batched
kernels run the same body on argument sets read from a table), for a mixed
set: 2D FP32 plans of different sizes and orders with uniform configurations
(which share kernels), FP64 plans, 1D, 3D, periodic, a masked plan and a
CFL-10 plan whose strided sweeps take the exact two-pass path (both run by
themselves at their position); two batched steps in a row, on a non-default
stream (the staging of the argument tables reused).  One plan is also checked
against the oracle.
"""
import numpy as np
import pytest

from gpu_common import check, dev, host
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


def _specs(molt):
    dom, mask, cross = W.star_domain(96, seed=3)
    U = molt.UNIFORM_CONFIG
    return [
        dict(shape=(64, 64), h=1 / 63, bc=0, P=2, cfl=2.0, dtype="f32", flags=U),
        dict(shape=(100, 80), h=(1 / 79, 1 / 99), bc=0, P=2, cfl=2.0, dtype="f32", flags=U),
        dict(shape=(257, 130), h=(1 / 129, 1 / 256), bc=0, P=1, cfl=1.5, dtype="f32", flags=U),
        dict(shape=(130, 257), h=(1 / 256, 1 / 129), bc=0, P=3, cfl=2.0, dtype="f32", flags=U),
        dict(shape=(96, 64), h=1 / 64, bc=1, P=2, cfl=2.0, dtype="f32", flags=U),
        dict(shape=(200, 150), h=(1 / 149, 1 / 199), bc=0, P=2, cfl=2.0, dtype="f64"),
        dict(shape=(1000,), h=1 / 999, bc=0, P=3, cfl=2.0, dtype="f64"),
        dict(shape=(20, 24, 28), h=(1 / 27, 1 / 23, 1 / 19), bc=0, P=2, cfl=2.0, dtype="f32"),
        dict(shape=(96, 96), h=1 / 95, bc=0, P=2, cfl=1.5, dtype="f32", mask=mask, cross=cross),
        dict(shape=(300, 200), h=(1 / 199, 1 / 299), bc=0, P=2, cfl=10.0, dtype="f32"),
    ]


def _fields(torch, spec, seed):
    shape = spec["shape"]
    dirichlet = () if spec["bc"] == 1 else tuple(range(len(shape)))
    u0 = W.random_field(shape, seed=seed, dirichlet_axes=dirichlet)
    u1 = W.random_field(shape, seed=seed + 1, dirichlet_axes=dirichlet)
    if "mask" in spec:
        u0 = u0 * spec["mask"]
        u1 = u1 * spec["mask"]
    return dev(torch, u0, spec["dtype"]), dev(torch, u1, spec["dtype"])


def test_step_batch_equals_steps(torch_cuda, molt):
    torch = torch_cuda
    specs = _specs(molt)
    plans = [molt.Plan(**sp) for sp in specs]
    # two sets of buffers: batched and one-by-one
    a, b = zip(*[_fields(torch, sp, 500 + 7 * i) for i, sp in enumerate(specs)])
    a, b = list(a), list(b)
    a2, b2 = [t.clone() for t in a], [t.clone() for t in b]
    c = [torch.full_like(t, float("nan")) for t in a]
    c2 = [torch.full_like(t, float("nan")) for t in a]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(2):
            molt.step_batch(plans, a, b, c)
            for p, x, y, z in zip(plans, a2, b2, c2):
                p.step(x, y, z)
            a, b, c = b, c, a
            a2, b2, c2 = b2, c2, a2
    torch.cuda.synchronize()
    for sp, x, y in zip(specs, b, b2):
        gx, gy = host(x), host(y)
        same = np.array_equal(gx, gy)
        print("%s %s P=%d cfl=%g: batched == one by one: %s" % (sp["shape"], sp["dtype"], sp["P"], sp["cfl"], same))
        assert same, sp["shape"]
    # the first plan against the oracle: two steps from the same fields
    import oracle
    sp = specs[5]
    p0 = plans[5]
    u0, u1 = _fields(torch, sp, 500 + 7 * 5)
    pb = oracle.Problem(sp["shape"], sp["h"], sp["bc"], p0.info["alpha"])
    r1 = pb.step(host(u0), host(u1), sp["P"], p0.info["beta"])
    r2 = pb.step(host(u1), r1, sp["P"], p0.info["beta"])
    check("mol_step_batch 2 steps (200, 150) FP64 vs oracle", host(b[5]), r2, "f64")
    for p in plans:
        p.close()


def test_step_batch_errors(torch_cuda, molt):
    torch = torch_cuda
    p = molt.Plan((64, 64), 1 / 63, 0, P=2, cfl=2.0, dtype="f64")
    x = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    y, z = torch.zeros_like(x), torch.zeros_like(x)
    with pytest.raises(molt.MolError):
        molt.step_batch([p, p], [x, y], [y, x], [z, z])       # plans must be distinct
    with pytest.raises(molt.MolError):
        molt.step_batch([p], [x], [y], [y])                   # u_next overlaps u_curr
    molt.step_batch([], [], [], [])                           # an empty batch is fine
    p.close()
