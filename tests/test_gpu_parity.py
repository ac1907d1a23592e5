"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerances: 1e-12 for FP64, 1e-5 for FP32, both as relative L2 over the
field and per element (max |got - ref| / max |ref|); FP32 inputs are the FP64
inputs rounded, the oracle runs in FP64.  Every comparison prints both.

Single operators and single steps are compared with the FP64 oracle.  Runs of
many steps are compared with the 80-bit build of the same oracle source: the
literal D = v - L^{-1} v of the FP64 build loses digits to cancellation on
smooth data and the three-level recurrence accumulates them (1.9e-11 after the
200 steps of the 1D standing-mode case, against 8e-15 for the 80-bit build,
both measured against the exact closed form).
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


# (shape, h, bc, cfl) -- ragged sizes, lines longer than one strided tile,
# periodic and mixed boundary types
CASES = [
    ((37,), 1.0 / 36, 0, 2.0),
    ((1024,), 1.0 / 1023, 0, 2.0),
    ((64,), 1.0 / 64, 1, 1.3),
    ((45, 33), 1.0 / 32, 0, 2.0),
    ((70, 130), (1.0 / 129, 1.0 / 69), 0, 1.5),
    ((600, 200), (1.0 / 199, 1.0 / 599), 0, 2.0),
    ((96, 64), (1.0 / 64, 1.0 / 96), 1, 2.0),
    ((48, 80), (1.0 / 80, 1.0 / 47), (1, 0), 3.0),
    ((20, 24, 28), (1.0 / 27, 1.0 / 23, 1.0 / 19), 0, 2.0),
    ((16, 16, 16), 1.0 / 16, 1, 2.0),
    ((300, 12, 20), 1.0 / 50, (0, 0, 1), 2.0),
]


def _prob(oracle_mod, shape, h, bc, alpha):
    return oracle_mod.Problem(shape, h, bc, alpha)


def _dirichlet_axes(shape, bc):
    nd = len(shape)
    bb = list(bc) if np.ndim(bc) else [bc] * nd
    return tuple(a for a in range(nd) if bb[a] == 0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_operators(torch_cuda, molt, oracle_mod, case, dtype):
    torch = torch_cuda
    shape, h, bc, cfl = CASES[case]
    nd = len(shape)
    P = 2
    plan = molt.Plan(shape, h, bc, P=P, cfl=cfl, dtype=dtype)
    alpha = plan.info["alpha"]
    pb = _prob(oracle_mod, shape, h, bc, alpha)
    v = W.random_field(shape, seed=10 + case, dirichlet_axes=_dirichlet_axes(shape, bc))
    vd = dev(torch, v, dtype)
    out = torch.empty_like(vd)
    print("case", case, shape, "bc", bc, "nu", plan.info["nu"][:nd])
    for ax in range(nd):
        plan.apply("linv_" + "xyz"[ax], vd, out)
        torch.cuda.synchronize()
        check("linv axis %d %s" % (ax, shape), host(out), pb.linv(v, ax), dtype)
        plan.apply("d_" + "xyz"[ax], vd, out)
        torch.cuda.synchronize()
        check("D axis %d %s" % (ax, shape), host(out), pb.Dg(v, ax), dtype)
    plan.apply("C", vd, out)
    torch.cuda.synchronize()
    check("C %s" % (shape,), host(out), pb.C(v), dtype)
    plan.apply("D", vd, out)
    torch.cuda.synchronize()
    check("D %s" % (shape,), host(out), pb.D(v), dtype)
    for P in (1, 2, 3):
        plan = molt.Plan(shape, h, bc, P=P, cfl=cfl, dtype=dtype)
        pbP = _prob(oracle_mod, shape, h, bc, plan.info["alpha"])
        plan.apply("rhs", vd, out)
        torch.cuda.synchronize()
        check("rhs P=%d %s" % (P, shape), host(out), pbP.rhs(v, P, plan.info["beta"]), dtype)
        plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("P", [1, 2, 3])
def test_step_and_start(torch_cuda, molt, oracle_mod, P, dtype):
    torch = torch_cuda
    shape, h = (90, 110), (1.0 / 109, 1.0 / 89)
    plan = molt.Plan(shape, h, 0, P=P, cfl=2.0, dtype=dtype)
    pb = oracle_mod.Problem(shape, h, 0, plan.info["alpha"])
    u0 = W.gaussian_pulses_2d(110, seed=P, npulses=3, sigma=0.05, ny=90)
    u1 = pb.start(u0, P, plan.info["beta"])
    d0, d1 = dev(torch, u0, dtype), dev(torch, u1, dtype)
    o = torch.empty_like(d0)
    plan.start(d0, o)
    torch.cuda.synchronize()
    check("start P=%d" % P, host(o), u1, dtype)
    plan.step(d0, d1, o)
    torch.cuda.synchronize()
    check("step P=%d" % P, host(o), pb.step(u0, u1, P, plan.info["beta"]), dtype)
    # u_next may alias u_prev
    plan.step(d0, d1, d0)
    torch.cuda.synchronize()
    check("step in place P=%d" % P, host(d0), pb.step(u0, u1, P, plan.info["beta"]), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nsteps,P", [(1, 2), (6, 2), (25, 2), (9, 3), (11, 1), (13, 4)])
def test_solve_graph(torch_cuda, molt, oracle_mod, dtype, nsteps, P):
    torch = torch_cuda
    shape, h = (64, 96), (1.0 / 95, 1.0 / 63)
    for flags in (0, molt.NO_GRAPH, molt.INCREMENT_FORM):
        plan = molt.Plan(shape, h, 0, P=P, cfl=2.0, dtype=dtype, flags=flags)
        pb = oracle_mod.Problem(shape, h, 0, plan.info["alpha"], precision="ld")
        u0 = W.gaussian_pulses_2d(96, seed=4, npulses=3, sigma=0.06, ny=64)
        u1 = pb.start(u0, P, plan.info["beta"])
        a, b = pb.run(u0, u1, nsteps, P, plan.info["beta"])
        da, db = dev(torch, u0, dtype), dev(torch, u1, dtype)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            plan.solve(da, db, nsteps)
        torch.cuda.synchronize()
        check("solve flags=%d n=%d prev" % (flags, nsteps), host(da), a, dtype)
        check("solve flags=%d n=%d curr" % (flags, nsteps), host(db), b, dtype)
        # a second call of 9 steps on the same buffers replays the captured
        # 8-step graph (captured by the first call when it held a whole unit)
        # and runs one more step
        with torch.cuda.stream(stream):
            plan.solve(da, db, 9)
        torch.cuda.synchronize()
        a2, b2 = pb.run(a, b, 9, P, plan.info["beta"])
        check("solve again flags=%d" % flags, host(db), b2, dtype)
        plan.close()


def test_config1_1d_full_run(torch_cuda, molt, oracle_mod):
    # 1D, N = 1024, Dirichlet, P = 1, CFL = 2, 200 steps, FP64
    torch = torch_cuda
    n = 1024
    h = 1.0 / (n - 1)
    x, u0, amps = W.sine_modes_1d(n, seed=1)
    plan = molt.Plan((n,), h, 0, P=1, cfl=2.0, dtype="f64")
    pb = oracle_mod.Problem((n,), h, 0, plan.info["alpha"], precision="ld")
    u1 = pb.start(u0, 1, plan.info["beta"])
    a, b = pb.run(u0, u1, 199, 1, plan.info["beta"])
    d0, d1 = dev(torch, u0, "f64"), dev(torch, u1, "f64")
    s = torch.empty_like(d0)
    plan.start(d0, s)
    plan.solve(d0, s, 199)
    torch.cuda.synchronize()
    check("config 1 u^200 vs 80-bit oracle", host(s), b, "f64")
    # and against the exact discrete closed form (sine modes are eigenvectors)
    import mpmath as mp
    import closed_forms as cf
    exact = np.zeros(n)
    for A, k in zip(amps, (1, 3)):
        Dh = 1 - cf.khat(mp.pi * k * h, plan.info["alpha"] * h)
        r = cf.rhs_symbol(1, plan.info["beta"], Dh, Dh)
        exact += float(A * cf.mode_sequence(r, 1, 1 + r / 2, 200)[200]) * np.sin(k * np.pi * x)
    exact[0] = exact[-1] = 0.0
    check("config 1 u^200 vs closed form", host(s), exact, "f64")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_split_tiles_long_columns(torch_cuda, molt, oracle_mod, dtype):
    # y lines of 2100 nodes: several strided tiles joined through the halo
    torch = torch_cuda
    shape, h = (2100, 70), 1.0 / 2099
    for cfl in (1.0, 2.0, 4.0):
        plan = molt.Plan(shape, h, 0, P=2, cfl=cfl, dtype=dtype)
        pb = oracle_mod.Problem(shape, h, 0, plan.info["alpha"])
        v = W.random_field(shape, 3, (0, 1))
        vd = dev(torch, v, dtype)
        o = torch.empty_like(vd)
        plan.apply("d_y", vd, o)
        torch.cuda.synchronize()
        check("D_y 2100 rows cfl=%g" % cfl, host(o), pb.Dg(v, 1), dtype)
        plan.apply("rhs", vd, o)
        torch.cuda.synchronize()
        check("rhs 2100 rows cfl=%g" % cfl, host(o), pb.rhs(v, 2, plan.info["beta"]), dtype)


# long y lines (several strips of the pipelined strided kernel, ragged last
# sub-tile, periodic wrap) and one long z line case
STRIP_CASES = [
    ((1100, 70), 1.0 / 1099, 0, 2.0),
    ((1100, 70), (1.0 / 70, 1.0 / 1100), (0, 1), 2.0),
    ((1024, 100), 1.0 / 1024, 1, 3.0),
    ((700, 130), 1.0 / 699, 0, 4.0),
    # small nu: exact two-pass sweeps of the L^{-1} form in both directions,
    # x lines of 4096 nodes (every x configuration the headline grid offers)
    ((1100, 70), 1.0 / 1099, 0, 100.0),
    ((96, 4096), 1.0 / 4095, 0, 100.0),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(STRIP_CASES)))
def test_every_strided_config(torch_cuda, molt, oracle_mod, case, dtype):
    # every valid configuration of every strided kernel of the fused solve
    # step, three steps against the 80-bit oracle
    torch = torch_cuda
    shape, h, bc, cfl = STRIP_CASES[case]
    plan = molt.Plan(shape, h, bc, P=2, cfl=cfl, dtype=dtype)
    pb = oracle_mod.Problem(shape, h, bc, plan.info["alpha"], precision="ld")
    u0 = W.random_field(shape, seed=20 + case, dirichlet_axes=_dirichlet_axes(shape, bc))
    u1 = pb.start(u0, 2, plan.info["beta"])
    a, b = pb.run(u0, u1, 3, 2, plan.info["beta"])
    nk = plan.info["kernels_per_step"]
    tried = 0
    for k in range(nk):
        ids, cur = plan.kernel_configs(k)
        for cfg in ids:
            plan.set_kernel_config(k, cfg)
            da, db = dev(torch, u0, dtype), dev(torch, u1, dtype)
            plan.solve(da, db, 3)
            torch.cuda.synchronize()
            check("strips %s kernel %d cfg %d" % (shape, k, cfg), host(db), b, dtype)
            tried += 1
        plan.set_kernel_config(k, cur)
    assert tried > 0
    plan.close()


# 3D: y lines of 300 nodes carry the two-combination sweeps of the box
# schedule, z lines of 280 the one-combination sweeps
BOX_STRIP_CASES = [
    ((24, 300, 40), (1.0 / 39, 1.0 / 299, 1.0 / 23), 0, 2.0),
    ((280, 30, 20), (1.0 / 19, 1.0 / 30, 1.0 / 280), (0, 1, 1), 2.0),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(BOX_STRIP_CASES)))
def test_every_strided_config_3d(torch_cuda, molt, oracle_mod, case, dtype):
    torch = torch_cuda
    shape, h, bc, cfl = BOX_STRIP_CASES[case]
    plan = molt.Plan(shape, h, bc, P=2, cfl=cfl, dtype=dtype)
    pb = oracle_mod.Problem(shape, h, bc, plan.info["alpha"], precision="ld")
    u0 = W.random_field(shape, seed=40 + case, dirichlet_axes=_dirichlet_axes(shape, bc))
    u1 = pb.start(u0, 2, plan.info["beta"])
    a, b = pb.run(u0, u1, 2, 2, plan.info["beta"])
    tried = 0
    for k in range(plan.info["kernels_per_step"]):
        ids, cur = plan.kernel_configs(k)
        for cfg in ids:
            plan.set_kernel_config(k, cfg)
            da, db = dev(torch, u0, dtype), dev(torch, u1, dtype)
            plan.solve(da, db, 2)
            torch.cuda.synchronize()
            check("box %s kernel %d cfg %d" % (shape, k, cfg), host(db), b, dtype)
            tried += 1
        plan.set_kernel_config(k, cur)
    assert tried > 0
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_long_z_lines(torch_cuda, molt, oracle_mod, dtype):
    torch = torch_cuda
    shape, h = (600, 12, 20), (1.0 / 19, 1.0 / 11, 1.0 / 599)     # z lines of 600 nodes
    plan = molt.Plan(shape, h, 0, P=2, cfl=2.0, dtype=dtype)
    pb = oracle_mod.Problem(shape, h, 0, plan.info["alpha"])
    v = W.random_field(shape, 5, (0, 1, 2))
    vd = dev(torch, v, dtype)
    o = torch.empty_like(vd)
    plan.apply("d_z", vd, o)
    torch.cuda.synchronize()
    check("D_z 600 planes", host(o), pb.Dg(v, 2), dtype)
    plan.apply("rhs", vd, o)
    torch.cuda.synchronize()
    check("rhs 600 planes", host(o), pb.rhs(v, 2, plan.info["beta"]), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("P", [4, 5])
def test_high_order_rhs_and_steps(torch_cuda, molt, oracle_mod, P, dtype):
    # orders 8 and 10 (Table 1 lists beta_max up to P = 5)
    torch = torch_cuda
    for shape, h, bc in (((200,), 1.0 / 199, 0), ((40, 56), (1.0 / 55, 1.0 / 39), 0),
                         ((36, 48), (1.0 / 48, 1.0 / 36), 1)):
        plan = molt.Plan(shape, h, bc, P=P, cfl=2.0, dtype=dtype)
        beta = plan.info["beta"]
        pb = oracle_mod.Problem(shape, h, bc, plan.info["alpha"])
        v = W.random_field(shape, seed=50 + P, dirichlet_axes=_dirichlet_axes(shape, bc))
        vd = dev(torch, v, dtype)
        out = torch.empty_like(vd)
        plan.apply("rhs", vd, out)
        torch.cuda.synchronize()
        check("rhs P=%d %s" % (P, shape), host(out), pb.rhs(v, P, beta), dtype)
        pl = oracle_mod.Problem(shape, h, bc, plan.info["alpha"], precision="ld")
        u1 = pl.start(v, P, beta)
        a, b = pl.run(v, u1, 4, P, beta)
        da, db = dev(torch, v, dtype), dev(torch, u1, dtype)
        plan.solve(da, db, 4)
        torch.cuda.synchronize()
        check("solve P=%d %s" % (P, shape), host(db), b, dtype)
        plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_minimum_sizes(torch_cuda, molt, oracle_mod, dtype):
    # the smallest grids a plan accepts: 3 nodes per axis
    torch = torch_cuda
    for shape, bc in (((3,), 0), ((3,), 1), ((3, 3), 0), ((3, 4), (1, 0)), ((3, 3, 3), 1),
                      ((5, 3, 4), 0)):
        nd = len(shape)
        bb = list(bc) if np.ndim(bc) else [bc] * nd
        h = tuple(1.0 / (shape[nd - 1 - a] - (0 if bb[a] else 1)) for a in range(nd))
        plan = molt.Plan(shape, h, bc, P=2, cfl=1.0, dtype=dtype)
        pb = oracle_mod.Problem(shape, h, bc, plan.info["alpha"])
        v = W.random_field(shape, seed=60, dirichlet_axes=_dirichlet_axes(shape, bc))
        vd = dev(torch, v, dtype)
        out = torch.empty_like(vd)
        plan.apply("rhs", vd, out)
        torch.cuda.synchronize()
        check("rhs %s bc %s" % (shape, bc), host(out), pb.rhs(v, 2, plan.info["beta"]), dtype,
              TOL[dtype] if np.linalg.norm(pb.rhs(v, 2, plan.info["beta"])) > 0 else 1e-30)
        plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_longest_x_lines(torch_cuda, molt, oracle_mod, dtype):
    # x lines of 16384 nodes (one workgroup of 16 waves): a step against the
    # FP64 oracle and 3 graph steps against the 80-bit oracle; Dirichlet P = 2
    # and periodic P = 3 (FP64 with two swept combinations does not fit the
    # LDS at this length: P = 3 runs in FP32 only)
    torch = torch_cuda
    cases = [((6, 16384), 1.0 / 16383, 0, 2)]
    if dtype == "f32":
        cases.append(((5, 16384), 1.0 / 16384, 1, 3))
    for shape, h, bc, P in cases:
        plan = molt.Plan(shape, h, bc, P=P, cfl=2.0, dtype=dtype)
        beta = plan.info["beta"]
        pb = oracle_mod.Problem(shape, h, bc, plan.info["alpha"])
        da = _dirichlet_axes(shape, bc)
        up = W.random_field(shape, seed=61, dirichlet_axes=da)
        uc = W.random_field(shape, seed=62, dirichlet_axes=da)
        a, b = dev(torch, up, dtype), dev(torch, uc, dtype)
        out = torch.empty_like(a)
        plan.step(a, b, out)
        torch.cuda.synchronize()
        check("step %s P=%d bc=%d" % (shape, P, bc), host(out), pb.step(up, uc, P, beta), dtype)
        pl = oracle_mod.Problem(shape, h, bc, plan.info["alpha"], precision="ld")
        ra, rb = pl.run(up, uc, 3, P, beta)
        plan.solve(a, b, 3)
        torch.cuda.synchronize()
        check("solve 3 %s P=%d bc=%d" % (shape, P, bc), host(b), rb, dtype)
        plan.close()
