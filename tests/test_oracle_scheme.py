"""Pins of the full scheme: Table 3, temporal order 2P, energy conservation and
no growth at CFL >> 1, the Table 2 operation count, commutation on
rectangles, 1D recovery, 3D plane waves, embedded line objects."""
import mpmath as mp
import numpy as np
import pytest

import closed_forms as cf
from conftest import golden
from oracle import lines, scheme
from paper_1308_3214_amd import workloads as W


def test_table3_closed_form_matches_printed():
    rows = golden("table3_adi_errors.txt")
    for row in rows:
        dt = float(row[0])
        for P in (1, 2, 3):
            printed = float(row[P])
            got = float(cf.table3_error(P, dt, scheme.beta_max(P)))
            if P == 1:
                # every printed digit
                assert float("%.2e" % got) == printed, (P, dt, got, printed)
            elif P == 2:
                assert abs(got / printed - 1) < 0.02, (P, dt, got, printed)
            else:
                assert abs(got / printed - 1) < 0.25, (P, dt, got, printed)


@pytest.mark.parametrize("P,dt", [(1, 0.1), (2, 0.2), (3, 0.4)])
def test_table3_time_stepped_equals_closed_form(oracle_mod, P, dt):
    u0, h = W.table3_mode(641)
    b = scheme.beta_max(P)
    pb = oracle_mod.Problem(u0.shape, h, oracle_mod.DIRICHLET, b / dt)
    om = np.sqrt(2) * np.pi
    a, c = u0, u0 * np.cos(om * dt)
    err = np.sqrt(h * h * ((c - u0 * np.cos(om * dt)) ** 2).sum())
    for s in range(2, int(round(1.2 / dt)) + 1):
        a, c = c, pb.step(a, c, P, b)
        err = max(err, np.sqrt(h * h * ((c - u0 * np.cos(om * s * dt)) ** 2).sum()))
    assert abs(err - float(cf.table3_error(P, dt, b))) < 1e-10


def test_temporal_order_2P(oracle_mod):
    # standing wave sin(2 pi x) on [0, 1] (Sec. 3.3) with a fine grid: the
    # error falls at rate 2P until the spatial floor
    n = 2001
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    u0 = np.sin(2 * np.pi * x)
    u0[0] = u0[-1] = 0.0
    for P, lo in ((1, 1.8), (2, 3.5), (3, 5.0)):
        b = scheme.beta_max(P)
        errs = []
        for dt in (0.1, 0.05, 0.025):
            pb = oracle_mod.Problem((n,), h, oracle_mod.DIRICHLET, b / dt)
            a, c = u0, u0 * np.cos(2 * np.pi * dt)
            e = 0.0
            for s in range(2, int(round(1.0 / dt)) + 1):
                a, c = c, pb.step(a, c, P, b)
                e = max(e, np.sqrt(h * ((c - u0 * np.cos(2 * np.pi * s * dt)) ** 2).sum()))
            errs.append(e)
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert (rates > lo).all() and (rates < 2 * P + 0.6).all(), (P, errs, rates)


@pytest.mark.parametrize("cfl", [10, 100, 1000])
def test_energy_conserved_no_growth(oracle_mod, cfl):
    # symmetric operators (uniform Dirichlet, periodic): the leapfrog energy
    # |u^{n+1} - u^n|^2 + <u^{n+1}, K u^n> with K u = -rhs(u) is conserved
    g = np.random.default_rng(cfl)
    for shape, bc in (((64,), 0), ((12, 16), (1, 0))):
        P = 2
        b = scheme.beta_max(P)
        h = 1.0 / 63 if len(shape) == 1 else (1.0 / 15, 1.0 / 12)
        hx = h if np.ndim(h) == 0 else h[0]
        pb = oracle_mod.Problem(shape, h, bc, b / (cfl * hx))
        u0 = W.random_field(shape, seed=cfl, dirichlet_axes=(0,) if len(shape) == 1 else (1,))
        u1 = pb.start(u0, P, b)

        def E(a, c):
            return float(np.sum((c - a) ** 2) + np.sum(c * -pb.rhs(a, P, b)))
        a, c = u0, u1
        E0 = E(a, c)
        mx = 0.0
        for _ in range(400 if len(shape) == 2 else 3000):
            a, c = c, pb.step(a, c, P, b)
            mx = max(mx, np.abs(c).max())
        assert abs(E(a, c) - E0) < 1e-12 * max(1.0, abs(E0))
        assert mx < 10 * np.abs(u0).max()


def test_table2_operation_count(oracle_mod):
    pb = oracle_mod.Problem((16, 16), 1.0 / 15, 0, 20.0)
    u = W.random_field((16, 16), 1, (0, 1))
    for P, expect in ((1, 1), (2, 3), (3, 6), (4, 10)):
        oracle_mod.count_reset()
        pb.rhs(u, P, scheme.beta_max(P))
        assert oracle_mod.count_get() == expect == P * (P + 1) // 2


def test_commutation_on_rectangles(oracle_mod):
    shape = (20, 28)
    h = (1.0 / 27, 1.0 / 19)
    for bc in (0, 1, (1, 0)):
        pb = oracle_mod.Problem(shape, h, bc, 30.0)
        v = W.random_field(shape, 5, () if bc == 1 else ((0, 1) if bc == 0 else (1,)))
        xy = pb.linv(pb.linv(v, 1), 0)
        yx = pb.linv(pb.linv(v, 0), 1)
        assert np.abs(xy - yx).max() < 1e-14
        # the D-form composition equals the literal operators
        Dx, Dy = pb.Dg(v, 0), pb.Dg(v, 1)
        DxDy = pb.Dg(Dy, 0)
        assert np.abs(pb.C(v) - (Dx + Dy - 2 * DxDy)).max() < 1e-14
        assert np.abs(pb.D(v) - (Dx + Dy - DxDy)).max() < 1e-14


def test_2d_with_y_independent_periodic_data_is_1d(oracle_mod):
    # Sec. 4: with C = D the ADI scheme is the 1D scheme
    nx, ny = 40, 8
    h = 1.0 / (nx - 1)
    u1d = W.random_field((nx,), 3, (0,))
    u2d = np.tile(u1d, (ny, 1))
    for P in (1, 2, 3):
        b = scheme.beta_max(P)
        p1 = oracle_mod.Problem((nx,), h, 0, b / (2 * h))
        p2 = oracle_mod.Problem((ny, nx), (h, 0.1), (0, 1), b / (2 * h))
        r1 = p1.rhs(u1d, P, b)
        r2 = p2.rhs(u2d, P, b)
        assert np.abs(r2 - r1[None, :]).max() < 1e-14


def test_3d_plane_waves_closed_form(oracle_mod):
    n = 12
    h = 1.0 / n
    ks = [(1, 2, 0), (3, -1, 2)]
    x = np.arange(n) * h
    P, cfl, nsteps = 2, 2.0, 12
    b = scheme.beta_max(P)
    alpha = b / (cfl * h)
    pb = oracle_mod.Problem((n, n, n), h, 1, alpha)
    modes = []
    for (kx, ky, kz), ph in zip(ks, (0.3, 1.1)):
        modes.append(np.cos(2 * np.pi * (kx * x[None, None, :] + ky * x[None, :, None]
                                         + kz * x[:, None, None]) + ph))
    u0 = modes[0] + 0.5 * modes[1]
    u1 = pb.start(u0, P, b)
    a, c = pb.run(u0, u1, nsteps - 1, P, b)
    expect = np.zeros_like(u0)
    for amp, (kx, ky, kz), md in zip((1.0, 0.5), ks, modes):
        Kg = [cf.khat(2 * mp.pi * k * h, alpha * h) for k in (kx, ky, kz)]
        Dg = [1 - K for K in Kg]
        Ch = Kg[1] * Kg[2] * Dg[0] + Kg[2] * Kg[0] * Dg[1] + Kg[0] * Kg[1] * Dg[2]
        Dh = 1 - Kg[0] * Kg[1] * Kg[2]
        r = cf.rhs_symbol(P, b, Ch, Dh)
        seq = cf.mode_sequence(r, 1, 1 + r / 2, nsteps)
        expect += amp * float(seq[nsteps]) * md
    assert np.abs(c - expect).max() < 1e-12


def test_line_objects_cover_the_mask():
    dom, mask, cross = W.star_domain(96, seed=2)
    for axis in (0, 1):
        idx, th = lines.extract(mask, cross, axis)
        cover = np.zeros_like(mask, dtype=np.int64)
        for (line, i0, i1) in idx:
            if axis == 0:
                cover[line, i0:i1 + 1] += 1
            else:
                cover[i0:i1 + 1, line] += 1
        assert (cover == mask).all()
        assert ((th > 0) & (th <= 1)).all()
    # every crossing lies on the curve
    h = 1.0 / 95
    jj, ii = np.nonzero(~np.isnan(cross[1]))
    px = ii * h + cross[1, jj, ii] * h
    r = np.hypot(px - 0.5, jj * h - 0.5)
    th = np.arctan2(jj * h - 0.5, px - 0.5)
    assert np.abs(r - dom.radius(th)).max() < 1e-12


def test_embedded_full_rectangle_reduces_to_dirichlet(oracle_mod):
    # a mask that is the whole interior of the grid with crossings on the ring
    # nodes gives exactly the rectangle operators
    ny, nx = 18, 23
    mask = np.zeros((ny, nx), np.uint8)
    mask[1:-1, 1:-1] = 1
    segs = lines.segments(mask, None)
    h = (1.0 / (nx - 1), 1.0 / (ny - 1))
    pe = oracle_mod.Problem((ny, nx), h, 0, 25.0, segments=segs, mask=mask)
    pr = oracle_mod.Problem((ny, nx), h, 0, 25.0)
    v = W.random_field((ny, nx), 9, (0, 1))
    for P in (1, 3):
        b = scheme.beta_max(P)
        assert np.abs(pe.rhs(v, P, b) - pr.rhs(v, P, b)).max() < 1e-14


def test_embedded_cavity_bounded(oracle_mod):
    # no growth on the (non-symmetric) embedded operators of the ellipse
    mask, cross = W.ellipse_domain(64)
    segs = lines.segments(mask, cross)
    n = 64
    h = 1.0 / (n - 1)
    P = 3
    b = scheme.beta_max(P)
    pb = oracle_mod.Problem((n, n), h, 0, b / (1.5 * h), segments=segs, mask=mask)
    x = np.arange(n) * h
    u0 = np.outer(np.exp(-(x - 0.5) ** 2 / 0.005), np.exp(-(x - 0.45) ** 2 / 0.005)) * mask
    a, c = pb.run(u0, pb.start(u0, P, b), 300, P, b)
    assert np.isfinite(c).all() and np.abs(c).max() < 2 * np.abs(u0).max()
    assert (c[mask == 0] == 0).all()


def test_long_run_reference_precision(oracle_mod):
    # 1D standing modes, N = 1024, P = 1, CFL = 2, 200 steps: both builds of
    # the oracle against the exact evolution of the two eigenmodes.  The FP64
    # build drifts (cancellation in D = v - L^{-1} v on smooth data); the
    # 80-bit build stays at rounding level and serves as the long-run reference.
    n = 1024
    h = 1.0 / (n - 1)
    x, u0, amps = W.sine_modes_1d(n, seed=1)
    P = 1
    b = scheme.beta_max(P)
    alpha = b / (2 * h)
    exact = np.zeros(n)
    for A, k in zip(amps, (1, 3)):
        Dh = 1 - cf.khat(mp.pi * k * h, alpha * h)
        r = cf.rhs_symbol(P, b, Dh, Dh)
        exact += float(A * cf.mode_sequence(r, 1, 1 + r / 2, 200)[200]) * np.sin(k * np.pi * x)
    exact[0] = exact[-1] = 0.0
    errs = {}
    for prec in ("f64", "ld"):
        pb = oracle_mod.Problem((n,), h, 0, alpha, precision=prec)
        _, c = pb.run(u0, pb.start(u0, P, b), 199, P, b)
        errs[prec] = np.linalg.norm(c - exact) / np.linalg.norm(exact)
    assert errs["ld"] < 5e-14, errs
    assert errs["f64"] < 1e-9, errs
