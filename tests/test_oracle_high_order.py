"""Pins of the orders 8 and 10 (P = 4, 5; Table 1 lists beta_max up to P = 5).

* The stage coefficients c_{p,m} of eq. Full_2D with the continuous symbol of
  L^{-1} (1 / (1 + k^2 / alpha^2), no spatial error) give temporal order 2P
  for P = 1..5 in the 40-digit recurrence of a standing wave.
* The oracle's step for P = 4, 5 on the sine mode (1D and 2D) equals the
  closed-form recurrence with the discrete symbol (kernel quadrature in
  mpmath), so the oracle carries those coefficients through Table 2's
  schedule without a dropped or misplaced term.
"""
import mpmath as mp
import numpy as np
import pytest

import closed_forms as cf
from oracle import scheme
from paper_1308_3214_amd import workloads as W


def _exact_symbol_error(P, dt, k=2 * mp.pi, T=1):
    b = mp.mpf(scheme.beta_max(P))
    dt = mp.mpf(dt)
    alpha = b / dt
    d = 1 - 1 / (1 + (k / alpha) ** 2)
    r = cf.rhs_symbol(P, b, d, d)           # 1D: C = D
    ns = int(mp.nint(T / dt))
    s = cf.mode_sequence(r, 1, mp.cos(k * dt), ns)
    return max(abs(s[j] - mp.cos(k * j * dt)) for j in range(1, ns + 1))


def test_stage_coefficients_give_order_2P():
    for P in range(1, 6):
        e = [_exact_symbol_error(P, dt) for dt in (0.05, 0.025, 0.0125)]
        rates = [float(mp.log(e[i] / e[i + 1], 2)) for i in range(2)]
        print("P=%d rates %s" % (P, rates))
        assert 2 * P - 0.6 < rates[-1] < 2 * P + 0.3, (P, rates)


@pytest.mark.parametrize("ndim,n,P", [(1, 41, 4), (1, 41, 5), (2, 33, 4), (2, 33, 5)])
def test_oracle_high_order_step_on_the_mode(oracle_mod, ndim, n, P):
    phi, h = W.sine_mode(n, ndim)
    dt = 0.05
    beta = scheme.beta_max(P)
    pb = oracle_mod.Problem(phi.shape, h, 0, beta / dt)
    Chat, Dhat = cf.mode_symbols(mp.mpf(h), mp.mpf(beta) / dt, ndim)
    r = cf.rhs_symbol(P, beta, Chat, Dhat)
    a0, a1 = 1.0, float(mp.cos(0.7 * dt))
    seq = cf.mode_sequence(r, a0, a1, 6)
    up, uc = a0 * phi, a1 * phi
    worst = 0.0
    for k in range(1, 6):
        up, uc = uc, pb.step(up, uc, P, beta)
        ref = float(seq[k + 1]) * phi
        worst = max(worst, np.abs(uc - ref).max() / np.abs(ref).max())
    print("ndim %d P %d: oracle vs recurrence %.3e" % (ndim, P, worst))
    assert worst < 1e-12
