"""Non-homogeneous boundary data in 1D by inverse Lax-Wendroff (Sec. 3.2),
test infrastructure (see the package header: only tests/, the smoke check and
the CPU-baseline leg of bench.py use the oracle).

Dirichlet data.  Each D^p of the 1D scheme (eq. update_P) is taken as p
applications of D = 1 - L^{-1}; an application to w = D^{p-1} u needs, at
each end, the curvature of w (the quadratic of the end cell) and the value
L^{-1} w must take there.  Both are even derivatives of u at the end, which
the wave equation turns into time derivatives of the boundary data (Sec. 3.2):
(d_xx)^j u = (d_tt / c^2)^j u_L.  With X = d_xx / alpha^2 and
U_j = (X^j u)(a) = (dt / beta)^{2j} d_t^{2j} u_L (alpha = beta / (c dt)), the
operators are power series in X,
    D = -X (1 - X)^{-1},   L^{-1} = (1 - X)^{-1},
so that at an end (binom(m, k) = 0 for m < k)
    (D^{p-1} u)            = (-1)^{p-1} sum_j binom(j - 1, p - 2) U_j   (p >= 2; U_0 for p = 1)
    (L^{-1} D^{p-1} u)     = (-1)^{p-1} sum_j binom(j, p - 1) U_j
    (X D^{p-1} u)          = (-1)^{p-1} sum_j binom(j - 2, p - 2) U_j   (p >= 2; U_1 for p = 1)
truncated at j <= P (U_j is of order dt^{2j}; the scheme's error is of order
dt^{2P+2} per step).  The end values of w need no data: each application
writes D w = w - L^{-1} w at the end nodes, which is the value the next one
reads.  After the step the end nodes take the boundary data at t_{n+1}.

Neumann data (the paper: the same procedure with odd derivatives).  With
u_x(a, t) = g_L(t), the slopes (X^j u_x)(a) = V_j = (dt / beta)^{2j} d_t^{2j} g_L
follow from the same identity, and the same series give the slope of
w = D^{p-1} u at the end and the slope L^{-1} w must take there.  The end
nodes are unknowns; the end cell's quadratic passes through the end node and
its neighbour with the slope of w at the end, and L^{-1} is closed by
imposing the slope of the result: for the convolution of the interpolant,
(I^L + I^R)' = alpha (I^R - I^L), so W = I^L + I^R + A e^{-alpha (x - a)}
+ B e^{-alpha (b - x)} has W'(a) = alpha I^R(a) - alpha A + alpha mu B and
W'(b) = -alpha I^L(b) - alpha mu A + alpha B, mu = e^{-alpha (b - a)}.
``linv_slopes`` computes I^L and I^R itself (numpy: local integrals with
weights from Gauss-Legendre on the reference cell, the recurrences by a
linear filter), independent of the C oracle it is pinned against.
"""
from __future__ import annotations

from math import comb

import numpy as np
from scipy.signal import lfilter

from . import linv_line
from .scheme import A_p


def _binom(m: int, k: int) -> int:
    return comb(m, k) if (m >= 0 and k >= 0 and m >= k) else 0


def ilw_sequence(derivs, dt, beta):
    """U_j = (dt / beta)^{2j} d_t^{2j} u_L, j = 0..len(derivs)-1, from the even
    time derivatives of the boundary data at t_n."""
    r = (float(dt) / float(beta)) ** 2
    return np.array([float(d) * r ** j for j, d in enumerate(derivs)])


def pass_data(p: int, U, alpha: float):
    """(value of D^{p-1} u, curvature of D^{p-1} u, target of L^{-1} D^{p-1} u)
    at one end for application p = 1..P, from U_0..U_P."""
    P = len(U) - 1
    s = (-1.0) ** (p - 1)
    if p == 1:
        val = U[0]
        kap = U[1] if P >= 1 else 0.0
    else:
        val = s * sum(_binom(j - 1, p - 2) * U[j] for j in range(p - 1, P + 1))
        kap = s * sum(_binom(j - 2, p - 2) * U[j] for j in range(p, P + 1))
    tgt = s * sum(_binom(j, p - 1) * U[j] for j in range(p - 1, P + 1))
    return float(val), float(alpha) ** 2 * float(kap), float(tgt)


def rhs_dirichlet(u, h, alpha, P, beta, Ua, Ub):
    """sum_p A_p D^p u on the line of nodes j h (j = 0..M) whose end nodes hold
    the boundary data; each D applied with the end curvatures and L^{-1}
    targets of pass_data at both ends."""
    u = np.asarray(u, dtype=np.float64)
    x = np.arange(len(u)) * float(h)
    w = u.copy()
    out = np.zeros_like(u)
    for p in range(1, P + 1):
        _, ka, ta = pass_data(p, Ua, alpha)
        _, kb, tb = pass_data(p, Ub, alpha)
        w = w - linv_line(x, w, alpha, (ta, tb, ka, kb))
        out += float(A_p(p, beta)) * w
    return out


def step_dirichlet(u_prev, u_curr, h, alpha, P, beta, da, db, next_a, next_b, dt):
    """One step of eq. update_P with Dirichlet data: da, db = even time
    derivatives d_t^{2j} u_L(t_n), d_t^{2j} u_R(t_n) for j = 0..P;
    next_a, next_b = the data at t_{n+1} (written at the end nodes)."""
    Ua, Ub = ilw_sequence(da, dt, beta), ilw_sequence(db, dt, beta)
    u_curr = np.asarray(u_curr, dtype=np.float64)
    out = 2.0 * u_curr - np.asarray(u_prev, dtype=np.float64) + rhs_dirichlet(
        u_curr, h, alpha, P, beta, Ua, Ub)
    out[0], out[-1] = next_a, next_b
    return out


# ---------------------------------------------------------------------------
# Neumann data
# ---------------------------------------------------------------------------
_GX, _GW = np.polynomial.legendre.leggauss(30)


def _cell_weights(nu: float):
    """Weights (c_m, c_0, c_p) of the local integral over one cell of width h,
    int_0^h (alpha/2) e^{-alpha s} q(s) ds, q the quadratic through
    (-h, v_m), (0, v_0), (h, v_p); nu = alpha h.  Gauss-Legendre on pieces
    of the cell with nu * width <= 1."""
    pieces = max(1, int(np.ceil(nu)))
    c = np.zeros(3)
    for k in range(pieces):
        lo, hi = k / pieces, (k + 1) / pieces
        t = 0.5 * (hi - lo) * _GX + 0.5 * (hi + lo)
        wt = 0.5 * (hi - lo) * _GW * 0.5 * nu * np.exp(-nu * t)
        # Lagrange basis of the nodes -1, 0, 1 at t
        c[0] += np.dot(wt, 0.5 * t * (t - 1.0))
        c[1] += np.dot(wt, 1.0 - t * t)
        c[2] += np.dot(wt, 0.5 * t * (t + 1.0))
    return c


def _il_ir(v, h, alpha, ghost_a, ghost_b):
    """I^L and I^R on a uniform line of M + 1 nodes, the end cells' quadratics
    through the ghost values ghost_a (node -1) and ghost_b (node M + 1)."""
    v = np.asarray(v, dtype=np.float64)
    M = len(v) - 1
    nu = alpha * h
    cm, c0, cp = _cell_weights(nu)
    ve = np.concatenate(([ghost_a], v, [ghost_b]))      # ve[i + 1] = v_i
    # J^R_i over [x_i, x_{i+1}], quadratic centred at x_i (i = 0..M-1)
    JR = cm * ve[0:M] + c0 * ve[1:M + 1] + cp * ve[2:M + 2]
    # J^L_i over [x_{i-1}, x_i], quadratic centred at x_i (i = 1..M): mirrored
    JL = cm * ve[3:M + 3] + c0 * ve[2:M + 2] + cp * ve[1:M + 1]
    d = np.exp(-nu)
    IL = np.zeros(M + 1)
    IR = np.zeros(M + 1)
    # I^L_j = d I^L_{j-1} + J^L_j (I^L_0 = 0), I^R_j = d I^R_{j+1} + J^R_j (I^R_M = 0)
    IL[1:] = lfilter([1.0], [1.0, -d], JL)
    IR[:M] = lfilter([1.0], [1.0, -d], JR[::-1])[::-1]
    return IL, IR


def linv_slopes(v, h, alpha, slope_v, target, closure="neumann"):
    """L^{-1} v on a uniform line of nodes a + j h, j = 0..M, whose end cells
    take the slopes slope_v = (v'(a), v'(b)) of the data (ghost values
    v_{-1} = v_1 - 2 h v'(a), v_{M+1} = v_{M-1} + 2 h v'(b)), closed by the
    slopes target = (W'(a), W'(b)) of the result (closure "neumann"), or, for
    the pin against the C oracle, by its values (closure "dirichlet")."""
    v = np.asarray(v, dtype=np.float64)
    M = len(v) - 1
    ga = v[1] - 2.0 * h * slope_v[0]
    gb = v[M - 1] + 2.0 * h * slope_v[1]
    IL, IR = _il_ir(v, h, alpha, ga, gb)
    mu = np.exp(-alpha * h * M)
    x = np.arange(M + 1) * h
    ea = np.exp(-alpha * x)
    eb = np.exp(-alpha * (x[-1] - x))
    if closure == "neumann":
        mat = np.array([[-1.0, mu], [-mu, 1.0]])
        rhs = np.array([target[0] / alpha - IR[0], target[1] / alpha + IL[M]])
    else:
        mat = np.array([[1.0, mu], [mu, 1.0]])
        rhs = np.array([target[0] - IR[0], target[1] - IL[M]])
    A, B = np.linalg.solve(mat, rhs)
    return IL + IR + A * ea + B * eb


def rhs_neumann(u, h, alpha, P, beta, Va, Vb):
    """sum_p A_p D^p u on a line with Neumann data: D applied with the slopes
    of pass_data (its value series taken on the slopes V_j) at both ends."""
    w = np.asarray(u, dtype=np.float64).copy()
    out = np.zeros_like(w)
    for p in range(1, P + 1):
        sa, _, ta = pass_data(p, Va, alpha)
        sb, _, tb = pass_data(p, Vb, alpha)
        w = w - linv_slopes(w, h, alpha, (sa, sb), (ta, tb))
        out += float(A_p(p, beta)) * w
    return out


def step_neumann(u_prev, u_curr, h, alpha, P, beta, ga, gb, dt):
    """One step of eq. update_P with Neumann data: ga, gb = even time
    derivatives d_t^{2j} u_x(a, t_n), d_t^{2j} u_x(b, t_n), j = 0..P.  Every
    node, the end nodes included, takes the update."""
    Va, Vb = ilw_sequence(ga, dt, beta), ilw_sequence(gb, dt, beta)
    u_curr = np.asarray(u_curr, dtype=np.float64)
    return 2.0 * u_curr - np.asarray(u_prev, dtype=np.float64) + rhs_neumann(
        u_curr, h, alpha, P, beta, Va, Vb)
