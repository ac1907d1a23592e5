"""The paper's ADI refinement study (Table 3) on the GPU: sin(pi x) sin(pi y)
on [-1, 1]^2 with 641^2 nodes, T = 1.2, beta = beta_max(P), exact u^1, FP64
plans through the C-ABI.  The max-over-steps discrete L2 error must equal the
closed-form value of the discrete scheme (a 40-digit single-mode evolution,
itself pinned to the printed Table 3 in test_oracle_scheme.py), i.e. the GPU
reproduces the printed errors: P = 1 to every digit, P = 2 within 2 %, P = 3
within 25 % (the closed form's agreement with the print)."""
import numpy as np
import pytest

import closed_forms as cf
from oracle import scheme
from paper_1308_3214_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("P,dt", [(1, 0.025), (2, 0.025), (3, 0.025), (2, 0.1), (3, 0.2)])
def test_table3_on_gpu(torch_cuda, P, dt):
    torch = torch_cuda
    from paper_1308_3214_amd import molt
    u0, h = W.table3_mode(641)
    om = np.sqrt(2.0) * np.pi
    nsteps = int(round(1.2 / dt))
    plan = molt.Plan(u0.shape, h, 0, P=P, dt=dt, dtype="f64")
    assert abs(plan.info["beta"] - scheme.beta_max(P)) < 1e-12
    ex = torch.tensor(u0, dtype=torch.float64, device="cuda")
    a = ex.clone()
    b = torch.tensor(u0 * np.cos(om * dt), dtype=torch.float64, device="cuda")
    err = 0.0
    for s in range(2, nsteps + 1):
        plan.solve(a, b, 1)
        torch.cuda.synchronize()
        err = max(err, float(torch.sqrt(h * h * ((b - ex * np.cos(om * s * dt)) ** 2).sum())))
    plan.close()
    ref = float(cf.table3_error(P, dt, scheme.beta_max(P)))
    print("Table 3 P=%d dt=%g: GPU max L2 error %.6e, closed form %.6e" % (P, dt, err, ref))
    assert abs(err / ref - 1) < 1e-8, (P, dt, err, ref)
