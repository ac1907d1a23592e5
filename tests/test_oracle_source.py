"""Pins of the oracle's step with a source term (Sec. 4, inclusion of source
terms).

* The reading of the C[S^n] coefficient is pinned by the order of accuracy
  against the exact solution of the forced wave equation: with the derived
  coefficient -beta^2 (c dt)^2 / 12 the P = 2 scheme converges at order 4 in
  dt (as the homogeneous scheme does in Table 3), with the printed one at
  order 2; P = 1 converges at order 2.  All in 40-digit closed form on the
  Table 3 grid (symbols from quadrature of the kernel, no oracle code).
* The oracle's step_source on the sine mode in 1D, 2D and 3D reproduces that
  closed-form scalar recurrence: a dropped term, a wrong sign or a swapped
  time level of S fails it.
"""
import mpmath as mp
import numpy as np
import pytest

import closed_forms as cf
from oracle import scheme
from paper_1308_3214_amd import workloads as W


def _orders(errs):
    return [float(mp.log(errs[i] / errs[i + 1], 2)) for i in range(len(errs) - 1)]


DTS = (0.1, 0.05, 0.025)


def test_source_order_pins_the_reading():
    e1 = [cf.forced_mode_error(1, dt, scheme.beta_max(1)) for dt in DTS]
    e2 = [cf.forced_mode_error(2, dt, scheme.beta_max(2)) for dt in DTS]
    e2p = [cf.forced_mode_error(2, dt, scheme.beta_max(2), coef="printed") for dt in DTS]
    o1, o2, o2p = _orders(e1), _orders(e2), _orders(e2p)
    print("P=1 orders", o1, "P=2 derived", o2, "P=2 printed", o2p)
    assert all(1.8 < o < 2.2 for o in o1), o1
    assert all(o > 3.7 for o in o2), o2
    assert all(o < 2.4 for o in o2p), o2p
    assert float(e2[-1]) < 1e-4 < float(e2p[-1])


W0 = 2.0


def _g(t):
    return (2 * mp.pi ** 2 - W0 ** 2) * mp.cos(W0 * t)    # any smooth g serves


@pytest.mark.parametrize("ndim,n,P", [(1, 41, 1), (1, 41, 2), (2, 41, 1), (2, 41, 2),
                                      (3, 17, 1), (3, 17, 2)])
def test_oracle_step_source_on_the_mode(oracle_mod, ndim, n, P):
    phi, h = W.sine_mode(n, ndim)
    dt = 0.08
    beta = scheme.beta_max(P)
    alpha = beta / dt
    pb = oracle_mod.Problem(phi.shape, h, 0, alpha)
    nsteps = 6
    a0, a1 = 1.0, float(mp.cos(W0 * dt))
    seq = cf.forced_mode_sequence(P, beta, dt, h, ndim, _g, a0, a1, nsteps)
    up, uc = a0 * phi, a1 * phi
    worst = 0.0
    for k in range(1, nsteps):
        t = k * dt
        un = pb.step_source(up, uc, float(_g(t - dt)) * phi, float(_g(t)) * phi,
                            float(_g(t + dt)) * phi, P, beta)
        ref = float(seq[k + 1]) * phi
        worst = max(worst, np.abs(un - ref).max() / np.abs(ref).max())
        up, uc = uc, un
    print("ndim %d P %d: oracle vs closed-form mode recurrence %.3e" % (ndim, P, worst))
    assert worst < 1e-12


def test_source_free_step_is_the_plain_step(oracle_mod):
    # S = 0: the step with a source is the homogeneous step exactly
    rng = np.random.default_rng(3)
    shape = (33, 40)
    pb = oracle_mod.Problem(shape, 1.0 / 39, 0, 30.0)
    up, uc = rng.standard_normal(shape), rng.standard_normal(shape)
    z = np.zeros(shape)
    for P in (1, 2):
        b = scheme.beta_max(P)
        assert np.array_equal(pb.step_source(up, uc, z, z, z, P, b), pb.step(up, uc, P, b))
    with pytest.raises(ValueError):
        pb.step_source(up, uc, z, z, z, 3, scheme.beta_max(3))


def test_source_step_keeps_dirichlet_nodes_zero(oracle_mod):
    # a source that is nonzero on the boundary does not move a Dirichlet node
    # (x Dirichlet, y periodic here)
    rng = np.random.default_rng(4)
    shape = (24, 17)
    pb = oracle_mod.Problem(shape, (1.0 / 16, 1.0 / 24), (0, 1), 25.0)
    f = [rng.standard_normal(shape) for _ in range(5)]
    for P in (1, 2):
        out = pb.step_source(*f, P, scheme.beta_max(P))
        assert np.all(out[:, 0] == 0) and np.all(out[:, -1] == 0)
        assert np.all(out[0, 1:-1] != 0)
