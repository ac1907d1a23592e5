"""Closed forms that pin the oracle (independent of its code).

* ``khat(theta, nu)``: the Fourier symbol of the discrete L^{-1} on a uniform
  grid.  For v_j = e^{i theta j} the left local integral is
  e^{i theta j} (nu/2) int_0^1 e^{-nu z} q(z) dz with q the Lagrange quadratic
  through (1, e^{-i theta}), (0, 1), (-1, e^{i theta}); the left recurrence
  sums the geometric series 1/(1 - d e^{-i theta}), d = e^{-nu}; the right
  half is the complex conjugate.  Evaluated with mpmath quadrature in 40
  digits: no closed-form weight is shared with the oracle.
* ``mode_max_error``: the three-level scheme acting on one eigenmode is a
  scalar recurrence a_{n+1} = (2 + r) a_n - a_{n-1}.
* ``forced_mode_*``: the same with a source S = g(t) phi on the mode phi:
  a_{n+1} = (2 + r) a_n - a_{n-1} + (source of the step acting on g).
"""
from __future__ import annotations

from math import comb, factorial

import mpmath as mp

mp.mp.dps = 40


def khat(theta, nu):
    with mp.workdps(40):
        return +_khat(theta, nu)


def _khat(theta, nu):
    theta = mp.mpf(theta)
    nu = mp.mpf(nu)
    em = mp.expj(-theta)
    ep = mp.expj(theta)

    def q(z):
        return em * z * (z + 1) / 2 + (1 - z * z) + ep * z * (z - 1) / 2

    JL = nu / 2 * mp.quad(lambda z: mp.exp(-nu * z) * q(z), [0, 1])
    d = mp.exp(-nu)
    return 2 * mp.re(JL / (1 - d * em))


def rhs_symbol(P, beta, Chat, Dhat):
    """sum_{p<=P} sum_{m<=p} (-1)^m 2 beta^{2m}/(2m)! binom(p-1,m-1) Chat^m Dhat^{p-m}
    (eq. Full_2D), with exact integer binomials and factorials."""
    beta = mp.mpf(beta)
    s = mp.mpf(0)
    for p in range(1, P + 1):
        for m in range(1, p + 1):
            s += (-1) ** m * 2 * beta ** (2 * m) / factorial(2 * m) * comb(p - 1, m - 1) \
                * Chat ** m * Dhat ** (p - m)
    return s


def mode_sequence(r, a0, a1, nsteps):
    """a_0, a_1, ..., a_nsteps of a_{n+1} = (2 + r) a_n - a_{n-1}."""
    out = [mp.mpf(a0), mp.mpf(a1)]
    for _ in range(nsteps - 1):
        out.append((2 + r) * out[-1] - out[-2])
    return out


def table3_error(P, dt, beta, n=641, T=1.2):
    """Max over steps n >= 1 of the discrete L2 error of the 2D ADI scheme for
    sin(pi x) sin(pi y) on [-1,1]^2 with n^2 nodes, u^1 exact.  The discrete L2
    norm of the mode on this node set is exactly 1 (sum of sin^2 over 640
    equispaced nodes of two periods = 320, times h = 2/640)."""
    h = mp.mpf(2) / (n - 1)
    dt = mp.mpf(dt)
    alpha = mp.mpf(beta) / dt
    Dx = 1 - khat(mp.pi * h, alpha * h)
    Kx = 1 - Dx
    Chat = Kx * Dx + Kx * Dx          # L_y^{-1} D_x + L_x^{-1} D_y
    Dhat = 1 - Kx * Kx                # 1 - L_x^{-1} L_y^{-1}
    r = rhs_symbol(P, beta, Chat, Dhat)
    om = mp.sqrt(2) * mp.pi
    ns = int(mp.nint(mp.mpf(T) / dt))
    seq = mode_sequence(r, 1, mp.cos(om * dt), ns)
    return max(abs(seq[k] - mp.cos(om * k * dt)) for k in range(1, ns + 1))


def mode_symbols(h, alpha, ndim):
    """(Chat, Dhat) of the sine mode sin(pi x) ... on [-1, 1]^ndim with spacing
    h in every direction: directional symbol d = 1 - khat(pi h, alpha h);
    1D: C = D = d; 2D: C = 2d - 2d^2, D = 2d - d^2; 3D: C = 3d - 6d^2 + 3d^3,
    D = 3d - 3d^2 + d^3 (the ADI compositions of equal directional symbols)."""
    d = 1 - khat(mp.pi * h, alpha * h)
    if ndim == 1:
        return d, d
    if ndim == 2:
        return 2 * d - 2 * d ** 2, 2 * d - d ** 2
    return 3 * d - 6 * d ** 2 + 3 * d ** 3, 3 * d - 3 * d ** 2 + d ** 3


def forced_source(P, beta, alpha, Chat, g_prev, g, g_next, coef="derived"):
    """Source part of one step acting on S = g phi.  coef = "derived":
    -beta^2 (c dt)^2 / 12 C[S^n]; coef = "printed": +beta^2 / (12 alpha^4) C[S^n]."""
    beta = mp.mpf(beta)
    a2 = (beta / alpha) ** 2
    if P == 1:
        return a2 * g
    s = a2 / 12 * (g_next + 10 * g + g_prev)
    if coef == "derived":
        return s - beta ** 2 * a2 / 12 * Chat * g
    return s + beta ** 2 / (12 * alpha ** 4) * Chat * g


def forced_mode_sequence(P, beta, dt, h, ndim, gfun, a0, a1, nsteps, coef="derived"):
    """a_0 .. a_nsteps of the scheme with source g(t) phi on the sine mode."""
    dt = mp.mpf(dt)
    alpha = mp.mpf(beta) / dt
    Chat, Dhat = mode_symbols(mp.mpf(h), alpha, ndim)
    r = rhs_symbol(P, beta, Chat, Dhat)
    out = [mp.mpf(a0), mp.mpf(a1)]
    for k in range(1, nsteps):
        t = k * dt
        src = forced_source(P, beta, alpha, Chat, gfun(t - dt), gfun(t), gfun(t + dt), coef)
        out.append((2 + r) * out[-1] - out[-2] + src)
    return out


def forced_mode_error(P, dt, beta, coef="derived", n=641, T=1.2, w0=2):
    """Max over steps of |a_n - A(t_n)| for the forced mode A(t) = cos(w0 t) of
    u_tt = laplacian(u) + S on [-1, 1]^2 (c = 1): S = (2 pi^2 - w0^2) cos(w0 t)
    sin(pi x) sin(pi y), u^0, u^1 exact, n^2 nodes (the Table 3 grid)."""
    h = mp.mpf(2) / (n - 1)
    g = lambda t: (2 * mp.pi ** 2 - w0 ** 2) * mp.cos(w0 * t)
    ns = int(mp.nint(mp.mpf(T) / dt))
    seq = forced_mode_sequence(P, beta, dt, h, 2, g, 1, mp.cos(w0 * mp.mpf(dt)), ns, coef)
    return max(abs(seq[k] - mp.cos(w0 * k * mp.mpf(dt))) for k in range(1, ns + 1))


def start_symbol_b(P, beta, Chat, Dhat):
    """sum_{p<=P} sum_{m<=p} (-1)^m beta^{2m}/(2m+1)! binom(p-1,m-1) Chat^m Dhat^{p-m}:
    the odd part of the start (Sec. 3.2) on a mode, exact integers."""
    beta = mp.mpf(beta)
    s = mp.mpf(0)
    for p in range(1, P + 1):
        for m in range(1, p + 1):
            s += (-1) ** m * beta ** (2 * m) / factorial(2 * m + 1) * comb(p - 1, m - 1) \
                * Chat ** m * Dhat ** (p - m)
    return s


def started_mode_error(P, dt, beta, n=641, T=1.2):
    """Max over steps of the error of the 2D scheme for u = (cos(w t) + sin(w t))
    sin(pi x) sin(pi y) on the Table 3 grid (w = sqrt(2) pi, g = w phi) with u^1
    from the start formula instead of the exact value."""
    h = mp.mpf(2) / (n - 1)
    dt = mp.mpf(dt)
    alpha = mp.mpf(beta) / dt
    Chat, Dhat = mode_symbols(h, alpha, 2)
    r = rhs_symbol(P, beta, Chat, Dhat)
    w = mp.sqrt(2) * mp.pi
    a1 = 1 + r / 2 + dt * w * (1 + start_symbol_b(P, beta, Chat, Dhat))
    ns = int(mp.nint(mp.mpf(T) / dt))
    seq = mode_sequence(r, 1, a1, ns)
    return max(abs(seq[k] - mp.cos(w * k * dt) - mp.sin(w * k * dt)) for k in range(1, ns + 1))
