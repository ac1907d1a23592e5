"""GPU parity of the 1D step with time-dependent boundary data (Sec. 3.2,
inverse Lax-Wendroff end data) through mol_step_bdata, against the oracle's
step_dirichlet and step_neumann.

Dirichlet and Neumann lines alike:
* One step on random interiors and random end data (values or slopes and
  their even time derivatives), P = 1..3, FP64 and FP32, lines of one to
  several lanes' worth with a ragged tail, CFL 2 and 10: relative L2 and per
  element within the bar.
* Zero data: the same as the homogeneous mol_step.
* A standing wave whose end values (or slopes) move in time, stepped 40 times
  on the GPU with the exact data: every step within the bar of the oracle's
  step from the same state, and the final error against the exact solution
  the same as the oracle run's (the GPU reproduces the order-2P accuracy, not
  only the arithmetic of one step).
Neumann lines also: mol_step, D_x and L^{-1}_x with zero slopes against the
oracle, and 9 graph-replayed steps of mol_solve against the oracle stepped
9 times.
"""
import numpy as np
import pytest

from gpu_common import check, dev, host

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


def _q(a, dtype):
    return np.asarray(a, np.float32).astype(np.float64) if dtype == "f32" else np.asarray(a)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("P", [1, 2, 3])
@pytest.mark.parametrize("n,cfl", [(37, 2.0), (1024, 2.0), (5001, 2.0), (700, 10.0)])
def test_one_step_random_data(torch_cuda, molt, n, cfl, P, dtype):
    from oracle import boundary as B
    torch = torch_cuda
    h = 1.0 / (n - 1)
    pl = molt.Plan((n,), h, molt.DIRICHLET, P=P, cfl=cfl, dtype=dtype)
    alpha, beta = pl.info["alpha"], pl.info["beta"]
    dt = cfl * h
    g = np.random.default_rng(1000 * P + n)
    up, uc = _q(g.uniform(-1, 1, n), dtype), _q(g.uniform(-1, 1, n), dtype)
    da = [float(g.uniform(-1, 1)) * 9.0 ** j for j in range(P + 1)]
    db = [float(g.uniform(-1, 1)) * 9.0 ** j for j in range(P + 1)]
    uc[0], uc[-1] = _q(da[0], dtype), _q(db[0], dtype)
    na, nb = float(g.uniform(-1, 1)), float(g.uniform(-1, 1))
    ref = B.step_dirichlet(up, uc, h, alpha, P, beta, da, db, na, nb, dt)
    a, b = dev(torch, up, dtype), dev(torch, uc, dtype)
    out = torch.full_like(a, float("nan"))
    pl.step_bdata(a, b, out, da, db, na, nb)
    torch.cuda.synchronize()
    check("dirichlet data n=%d cfl=%g P=%d" % (n, cfl, P), host(out), ref, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_zero_data_is_mol_step(torch_cuda, molt, dtype):
    torch = torch_cuda
    n, P = 2000, 3
    pl = molt.Plan((n,), 1.0 / (n - 1), molt.DIRICHLET, P=P, cfl=2.0, dtype=dtype)
    g = np.random.default_rng(7)
    up, uc = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    up[0] = up[-1] = uc[0] = uc[-1] = 0.0
    a, b = dev(torch, up, dtype), dev(torch, uc, dtype)
    o1, o2 = torch.empty_like(a), torch.empty_like(a)
    pl.step(a, b, o1)
    pl.step_bdata(a, b, o2, [0.0] * (P + 1), [0.0] * (P + 1), 0.0, 0.0)
    torch.cuda.synchronize()
    check("zero Dirichlet data vs mol_step", host(o2), host(o1), dtype)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_moving_ends_standing_wave(torch_cuda, molt, P):
    from oracle import boundary as B
    torch = torch_cuda
    n, cfl, k, phi = 2001, 4.0, 2.5 * np.pi, 0.3
    h = 1.0 / (n - 1)
    dt = cfl * h
    x = np.arange(n) * h
    pl = molt.Plan((n,), h, molt.DIRICHLET, P=P, cfl=cfl, dtype="f64")
    alpha, beta = pl.info["alpha"], pl.info["beta"]

    def exact(t):
        return np.cos(k * t) * np.cos(k * x + phi)

    def data(t):
        da = [(-k * k) ** j * np.cos(k * t) * np.cos(phi) for j in range(P + 1)]
        db = [(-k * k) ** j * np.cos(k * t) * np.cos(k + phi) for j in range(P + 1)]
        return da, db, np.cos(k * (t + dt)) * np.cos(phi), np.cos(k * (t + dt)) * np.cos(k + phi)

    u = [dev(torch, exact(0.0), "f64"), dev(torch, exact(dt), "f64"), None]
    u[2] = torch.empty_like(u[0])
    oa, ob = exact(0.0), exact(dt)
    nsteps = 40
    for s in range(1, nsteps):
        da, db, na, nb = data(s * dt)
        pl.step_bdata(u[0], u[1], u[2], da, db, na, nb)
        torch.cuda.synchronize()
        got = host(u[2])
        one = B.step_dirichlet(host(u[0]), host(u[1]), h, alpha, P, beta, da, db, na, nb, dt)
        check("moving ends step %d P=%d" % (s, P), got, one, "f64")
        u = [u[1], u[2], u[0]]
        oa, ob = ob, B.step_dirichlet(oa, ob, h, alpha, P, beta, da, db, na, nb, dt)
    eg = np.abs(host(u[1]) - exact(nsteps * dt)).max()
    eo = np.abs(ob - exact(nsteps * dt)).max()
    print("P=%d error against the exact solution after %d steps: GPU %.6e oracle %.6e"
          % (P, nsteps, eg, eo))
    assert abs(eg - eo) <= 1e-3 * eo + 1e-13


# ---------------------------------------------------------------------------
# Neumann lines
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("P", [1, 2, 3])
@pytest.mark.parametrize("n,cfl", [(37, 2.0), (1024, 2.0), (5001, 2.0), (700, 10.0)])
def test_neumann_one_step_random_data(torch_cuda, molt, n, cfl, P, dtype):
    from oracle import boundary as B
    torch = torch_cuda
    h = 1.0 / (n - 1)
    pl = molt.Plan((n,), h, molt.NEUMANN, P=P, cfl=cfl, dtype=dtype)
    alpha, beta = pl.info["alpha"], pl.info["beta"]
    assert pl.info["unknowns"] == n
    dt = cfl * h
    g = np.random.default_rng(2000 * P + n)
    up, uc = _q(g.uniform(-1, 1, n), dtype), _q(g.uniform(-1, 1, n), dtype)
    ga = [float(g.uniform(-1, 1)) * 9.0 ** j for j in range(P + 1)]
    gb = [float(g.uniform(-1, 1)) * 9.0 ** j for j in range(P + 1)]
    ref = B.step_neumann(up, uc, h, alpha, P, beta, ga, gb, dt)
    a, b = dev(torch, up, dtype), dev(torch, uc, dtype)
    out = torch.full_like(a, float("nan"))
    pl.step_bdata(a, b, out, ga, gb)
    torch.cuda.synchronize()
    check("neumann data n=%d cfl=%g P=%d" % (n, cfl, P), host(out), ref, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_neumann_homogeneous_operators_step_and_solve(torch_cuda, molt, dtype):
    from oracle import boundary as B
    torch = torch_cuda
    n, P, cfl = 3001, 2, 3.0
    h = 1.0 / (n - 1)
    pl = molt.Plan((n,), h, molt.NEUMANN, P=P, cfl=cfl, dtype=dtype)
    alpha, beta = pl.info["alpha"], pl.info["beta"]
    g = np.random.default_rng(31)
    v = _q(g.uniform(-1, 1, n), dtype)
    vd = dev(torch, v, dtype)
    out = torch.empty_like(vd)
    lv = B.linv_slopes(v, h, alpha, (0.0, 0.0), (0.0, 0.0))
    pl.apply("linv_x", vd, out)
    torch.cuda.synchronize()
    check("neumann L^-1_x zero slopes", host(out), lv, dtype)
    pl.apply("d_x", vd, out)
    torch.cuda.synchronize()
    check("neumann D_x zero slopes", host(out), v - lv, dtype)
    # steps: mol_step, and 9 steps of mol_solve (one 8-step graph unit and a
    # tail) on a non-default stream, against the oracle stepped 9 times
    x = np.arange(n) * h
    u0 = _q(np.cos(3 * np.pi * x) + 0.5 * np.cos(7 * np.pi * x) + 0.2 * np.exp(-((x - 0.3) / 0.05) ** 2),
            dtype)
    z = [0.0] * (P + 1)
    u1 = _q(u0 + 0.5 * (B.step_neumann(u0, u0, h, alpha, P, beta, z, z, cfl * h) - u0), dtype)
    a, b = dev(torch, u0, dtype), dev(torch, u1, dtype)
    o = torch.empty_like(a)
    pl.step(a, b, o)
    torch.cuda.synchronize()
    check("neumann mol_step zero slopes", host(o), B.step_neumann(u0, u1, h, alpha, P, beta, z, z, cfl * h),
          dtype)
    ra, rb = u0.copy(), u1.copy()
    for _ in range(9):
        ra, rb = rb, B.step_neumann(ra, rb, h, alpha, P, beta, z, z, cfl * h)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pl.solve(a, b, 9)
    torch.cuda.synchronize()
    check("neumann mol_solve 9 steps prev", host(a), ra, dtype)
    check("neumann mol_solve 9 steps curr", host(b), rb, dtype)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_neumann_moving_slopes_standing_wave(torch_cuda, molt, P):
    from oracle import boundary as B
    torch = torch_cuda
    n, cfl, k, phi = 2001, 4.0, 2.5 * np.pi, 0.3
    h = 1.0 / (n - 1)
    dt = cfl * h
    x = np.arange(n) * h
    pl = molt.Plan((n,), h, molt.NEUMANN, P=P, cfl=cfl, dtype="f64")
    alpha, beta = pl.info["alpha"], pl.info["beta"]

    def exact(t):
        return np.cos(k * t) * np.cos(k * x + phi)

    def data(t):
        ga = [(-k * k) ** j * (-k * np.sin(phi)) * np.cos(k * t) for j in range(P + 1)]
        gb = [(-k * k) ** j * (-k * np.sin(k + phi)) * np.cos(k * t) for j in range(P + 1)]
        return ga, gb

    u = [dev(torch, exact(0.0), "f64"), dev(torch, exact(dt), "f64"), None]
    u[2] = torch.empty_like(u[0])
    oa, ob = exact(0.0), exact(dt)
    nsteps = 40
    for s in range(1, nsteps):
        ga, gb = data(s * dt)
        pl.step_bdata(u[0], u[1], u[2], ga, gb)
        torch.cuda.synchronize()
        got = host(u[2])
        one = B.step_neumann(host(u[0]), host(u[1]), h, alpha, P, beta, ga, gb, dt)
        check("neumann moving slopes step %d P=%d" % (s, P), got, one, "f64")
        u = [u[1], u[2], u[0]]
        oa, ob = ob, B.step_neumann(oa, ob, h, alpha, P, beta, ga, gb, dt)
    eg = np.abs(host(u[1]) - exact(nsteps * dt)).max()
    eo = np.abs(ob - exact(nsteps * dt)).max()
    print("P=%d error against the exact solution after %d steps: GPU %.6e oracle %.6e"
          % (P, nsteps, eg, eo))
    assert abs(eg - eo) <= 1e-3 * eo + 1e-13
