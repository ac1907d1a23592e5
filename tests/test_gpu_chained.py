"""GPU parity of the chained y sweep of the fused 2D P = 2 solve.

In FP32 the solve step of a 2D P = 2 plan takes both y sweeps of a step in one
launch (v1 = C u stays on chip) when the y lines are long enough.  These cases
check that launch, in every one of its configurations, against the 80-bit
oracle and against the same plan with the two y sweeps split
(MOL_SPLIT_Y): line lengths at the minimum of two sub-tiles, ragged lengths and
widths, several strips per line, periodic lines and CFL 1 to 4 (halo and walk
lengths change with nu = alpha h).
"""
import numpy as np
import pytest

from gpu_common import check
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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float32)


# (shape (ny, nx), h (hx, hy), bc (x, y), cfl); dt = cfl h_x / c, so nu_y =
# beta h_y / (cfl h_x) sets the halo of the y lines
CASES = [
    ((128, 64), 1.0 / 127, 0, 2.0),                    # two sub-tiles: one strip, no walk ends
    ((129, 65), (1.0 / 64, 1.0 / 128), 0, 2.0),        # ragged last sub-tile and column group
    ((1100, 70), 1.0 / 1099, 0, 2.0),                  # several strips per line
    ((1100, 70), 1.0 / 1099, (0, 1), 2.0),             # periodic y
    ((130, 40), 1.0 / 130, 1, 2.0),                    # periodic, shortest line accepted
    ((1024, 100), 1.0 / 1024, 1, 3.0),
    ((700, 130), 1.0 / 699, 0, 4.0),                   # long halo (small nu)
    ((4100, 33), 1.0 / 4099, 0, 1.0),                  # long lines, large nu
    ((64, 96), (1.0 / 95, 1.0 / 63), 0, 2.0),          # nu_y = 1.1: only the 32-row sub-tiles
]


def _dirichlet_axes(bc):
    bb = list(bc) if np.ndim(bc) else [bc] * 2
    return tuple(a for a in range(2) if bb[a] == 0)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_chained_y_sweep(torch_cuda, molt, oracle_mod, case):
    torch = torch_cuda
    shape, h, bc, cfl = CASES[case]
    plan = molt.Plan(shape, h, bc, P=2, cfl=cfl, dtype="f32")
    split = molt.Plan(shape, h, bc, P=2, cfl=cfl, dtype="f32", flags=molt.SPLIT_Y)
    assert plan.info["kernels_per_step"] == 2, "chained y launch not used"
    assert split.info["kernels_per_step"] == 3
    pb = oracle_mod.Problem(shape, h, bc, plan.info["alpha"], precision="ld")
    u0 = W.random_field(shape, seed=40 + case, dirichlet_axes=_dirichlet_axes(bc))
    u1 = pb.start(u0, 2, plan.info["beta"])
    # one 8-step graph unit on a non-default stream plus an odd tail of one
    # step launched directly
    nsteps = 9
    a, b = pb.run(u0, u1, nsteps, 2, plan.info["beta"])
    stream = torch.cuda.Stream()

    def run(p):
        da, db = dev(torch, u0), dev(torch, u1)
        with torch.cuda.stream(stream):
            p.solve(da, db, nsteps)
        torch.cuda.synchronize()
        return da.double().cpu().numpy(), db.double().cpu().numpy()

    ga, gb = run(plan)
    sa, sb = run(split)
    for name, got, ref in (("prev", ga, a), ("curr", gb, b)):
        check("chained %s %s bc=%s cfl=%g" % (shape, name, bc, cfl), got, ref, "f32")
    check("chained vs split y sweeps", gb, sb, "f32")

    # every valid configuration of the chained launch
    ids, cur = plan.kernel_configs(0)
    assert len(ids) >= 1
    for cfg in ids:
        plan.set_kernel_config(0, cfg)
        _, gb2 = run(plan)
        check("chained cfg %d" % cfg, gb2, b, "f32")
    plan.set_kernel_config(0, cur)
    plan.close()
    split.close()


def test_chained_not_taken(torch_cuda, molt):
    # short y lines and FP64 keep the split y sweeps (square cells: nu_y =
    # nu_x = 0.74, above the threshold of the L^{-1}-composed steps)
    for kw in (dict(shape=(48, 96), dtype="f32"), dict(shape=(1100, 70), dtype="f64")):
        shape = kw.pop("shape")
        plan = molt.Plan(shape, 1.0 / (shape[1] - 1), 0, P=2, cfl=2.0, **kw)
        assert plan.info["kernels_per_step"] == 3, kw
        plan.close()
    # small nu (0.0047 along y): C from L^{-1} and D sweeps, no chained launch
    # (4 per step)
    plan = molt.Plan((1100, 70), (1.0 / 69, 1.0 / 1099), 0, P=2, cfl=20.0, dtype="f32")
    assert plan.info["kernels_per_step"] == 4
    plan.close()
