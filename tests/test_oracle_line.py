"""Pins of the one-line convolution L^{-1} (Sec. 2): the recursion O1 against
the direct quadrature O2, exact data, the discrete Fourier symbol, symmetry."""
import mpmath as mp
import numpy as np
import pytest

import closed_forms as cf
from oracle import direct


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("nu", [1e-3, 0.05, 0.3, 0.742, 1.9, 2.1, 6.0])
def test_recursion_matches_direct_quadrature(oracle_mod, nu):
    g = np.random.default_rng(7)
    for trial in range(3):
        m = 14
        h = 1.0 / m
        x = np.arange(m + 1) * h
        # non-uniform end cells as on an embedded line object (Sec. 4.3), some tiny
        x[0] += (0.0, 0.4, 1.0 - 1e-7)[trial] * h
        x[-1] -= (0.0, 0.75, 1.0 - 1e-6)[trial] * h
        v = g.uniform(-1, 1, m + 1)
        v[0] = v[-1] = 0.0
        w1 = oracle_mod.linv_line(x, v, nu / h)
        w2 = direct.linv_line_direct(x, v, nu / h)
        assert _rel(w1, w2) < 1e-13


@pytest.mark.parametrize("alpha", [0.5, 8.0, 80.0])
def test_periodic_recursion_matches_direct(oracle_mod, alpha):
    g = np.random.default_rng(3)
    n = 12
    v = g.uniform(-1, 1, n)
    w1 = oracle_mod.linv_periodic_line(v, 1.0 / n, alpha)
    w2 = direct.linv_periodic_direct(v, 1.0 / n, alpha)
    assert _rel(w1, w2) < 1e-13


def test_quadratic_data_is_exact(oracle_mod):
    # L = 1 - d_xx/alpha^2 maps v + v''/alpha^2 to v for quadratic v, so with
    # the end values w = v + v''/alpha^2 and the data's curvature at the ends
    # (inverse Lax-Wendroff, Sec. 3.2) the discrete L^{-1} is exact.
    g = np.random.default_rng(11)
    for alpha in (0.7, 3.0, 40.0):
        x = np.sort(g.uniform(0, 1, 17))
        x[0], x[-1] = 0.0, 1.0
        c0, c1, c2 = g.uniform(-2, 2, 3)
        v = c0 + c1 * x + c2 * x * x
        ex = v + 2 * c2 / alpha ** 2
        w = oracle_mod.linv_line(x, v, alpha, (ex[0], ex[-1], 2 * c2, 2 * c2))
        assert np.abs(w - ex).max() < 1e-13


def test_exponential_data_second_order(oracle_mod):
    # v = e^{g x}: the exact solution of (1 - d_xx/alpha^2) w = v on [0, 1] with
    # w(0) = w(1) = 0 is v/(1 - g^2/alpha^2) + A e^{-alpha x} + B e^{-alpha (1-x)};
    # the discrete L^{-1} converges to it at least at second order in h.
    gam, alpha = 1.7, 6.0
    errs = []
    for m in (20, 40, 80, 160):
        x = np.linspace(0.0, 1.0, m + 1)
        v = np.exp(gam * x)
        part = v / (1 - gam ** 2 / alpha ** 2)
        ea, eb = np.exp(-alpha * x), np.exp(-alpha * (1 - x))
        A, B = np.linalg.solve([[ea[0], eb[0]], [ea[-1], eb[-1]]], [-part[0], -part[-1]])
        exact = part + A * ea + B * eb
        w = oracle_mod.linv_line(x, v, alpha, (0.0, 0.0, gam ** 2, gam ** 2 * np.exp(gam)))
        errs.append(np.abs(w - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (rates > 1.9).all(), (errs, rates)


@pytest.mark.parametrize("nu", [0.01, 0.742, 3.0])
def test_sine_modes_are_eigenvectors(oracle_mod, nu):
    # Uniform Dirichlet line: with zero curvature at the end nodes the odd
    # extension is exact, so sin(k pi x_j) is an eigenvector and the eigenvalue
    # is the free-space symbol at theta = k pi h.
    n = 48
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    for k in (1, 4, 17, n - 2):
        v = np.sin(k * np.pi * x)
        v[0] = v[-1] = 0.0
        w = oracle_mod.linv_line(x, v, nu / h)
        K = float(cf.khat(mp.pi * k * h, nu))
        assert np.abs(w - K * v).max() < 5e-15


def test_plane_waves_periodic(oracle_mod):
    n = 20
    h = 1.0 / n
    for nu in (0.05, 0.742):
        for k in (0, 1, 6, 10):
            v = np.cos(2 * np.pi * k * np.arange(n) / n + 0.4)
            w = oracle_mod.linv_periodic_line(v, h, nu / h)
            K = float(cf.khat(2 * mp.pi * k * h, nu))
            assert np.abs(w - K * v).max() < 5e-15


def test_symbol_range():
    # 0 < Khat <= 1 for every theta and nu (no growth at any CFL), Khat(0) = 1
    for nu in (1e-4, 0.01, 0.3, 1.0, 8.0, 64.0):
        assert abs(cf.khat(0, nu) - 1) < mp.mpf("1e-30")
        for i in range(0, 65):
            K = cf.khat(mp.pi * i / 64, nu)
            assert 0 < K <= 1 + mp.mpf("1e-30")


def test_interior_operator_symmetric(oracle_mod):
    n = 24
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    for nu in (0.1, 0.742, 2.5):
        M = np.zeros((n - 2, n - 2))
        for j in range(n - 2):
            e = np.zeros(n)
            e[j + 1] = 1.0
            M[:, j] = oracle_mod.linv_line(x, e, nu / h)[1:-1]
        assert np.abs(M - M.T).max() < 1e-15
        # and positive definite with spectrum in (0, 1]
        ev = np.linalg.eigvalsh(0.5 * (M + M.T))
        assert ev.min() > 0 and ev.max() <= 1 + 1e-14
