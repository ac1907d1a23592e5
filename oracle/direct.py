"""O2: the discrete convolution L^{-1} evaluated directly (test infrastructure).

For every target node x_j, sum over all cells the integral of the Green's
function (alpha/2) e^{-alpha |x_j - y|} (Sec. 2, eq. L_Inverse) against the
local interpolant of the data, then add the homogeneous solutions that impose
the end values.  Cells left of x_j use the quadratic centred on the cell's
right node, cells right of x_j the quadratic centred on the cell's left node
-- the node each exponential recurrence arrives at (Sec. 2).  At a Dirichlet
end node the interpolant is the straight line through the cell's two nodes
plus the prescribed curvature (inverse Lax-Wendroff, Sec. 3.2).

Every cell is integrated with 20-point Gauss-Legendre (split into pieces of
alpha*width <= 2); exponentials are evaluated directly.  There is no
recurrence and no closed-form quadrature weight, so agreement with O1 pins the
recurrences, the powers of e^{-alpha h} and the weights of O1.  O(M^2) work:
use only on short lines.
"""
from __future__ import annotations

import numpy as np

_GX, _GW = np.polynomial.legendre.leggauss(20)


def _interp_coeffs(x, v, i, kap_a, kap_b):
    """Interpolant attached to node i, returned as a callable of y."""
    m = len(x) - 1
    if 0 < i < m:
        xa, xb, xc = x[i - 1], x[i], x[i + 1]
        va, vb, vc = v[i - 1], v[i], v[i + 1]

        def q(y):  # Lagrange form through three nodes
            return (va * (y - xb) * (y - xc) / ((xa - xb) * (xa - xc))
                    + vb * (y - xa) * (y - xc) / ((xb - xa) * (xb - xc))
                    + vc * (y - xa) * (y - xb) / ((xc - xa) * (xc - xb)))
        return q
    if i == 0:
        xa, xb, va, vb, kap = x[0], x[1], v[0], v[1], kap_a
    else:
        xa, xb, va, vb, kap = x[m - 1], x[m], v[m - 1], v[m], kap_b

    def q(y):  # chord plus prescribed curvature
        return va + (vb - va) * (y - xa) / (xb - xa) + 0.5 * kap * (y - xa) * (y - xb)
    return q


def _cell_integral(f, a, b, alpha):
    pieces = max(1, int(np.ceil(alpha * (b - a) / 2.0)))
    edges = np.linspace(a, b, pieces + 1)
    s = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        y = 0.5 * (hi - lo) * _GX + 0.5 * (hi + lo)
        s += 0.5 * (hi - lo) * np.dot(_GW, f(y))
    return s


def linv_line_direct(x, v, alpha, bnd=(0.0, 0.0, 0.0, 0.0)):
    """L^{-1} v on the bounded line object with nodes x[0..m]; bnd = (ta, tb, ka, kb)."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    ta, tb, ka, kb = (float(t) for t in bnd)
    m = len(x) - 1
    quads = [_interp_coeffs(x, v, i, ka, kb) for i in range(m + 1)]
    IL = np.zeros(m + 1)
    IR = np.zeros(m + 1)
    for j in range(m + 1):
        xj = x[j]
        for i in range(1, j + 1):          # cell [x_{i-1}, x_i] left of x_j
            q = quads[i]
            IL[j] += _cell_integral(lambda y: 0.5 * alpha * np.exp(-alpha * (xj - y)) * q(y),
                                    x[i - 1], x[i], alpha)
        for i in range(j, m):              # cell [x_i, x_{i+1}] right of x_j
            q = quads[i]
            IR[j] += _cell_integral(lambda y: 0.5 * alpha * np.exp(-alpha * (y - xj)) * q(y),
                                    x[i], x[i + 1], alpha)
    # homogeneous solutions A e^{-alpha (x - a)} + B e^{-alpha (b - x)} with w(a)=ta, w(b)=tb
    ea = np.exp(-alpha * (x - x[0]))
    eb = np.exp(-alpha * (x[-1] - x))
    mat = np.array([[ea[0], eb[0]], [ea[-1], eb[-1]]])
    rhs = np.array([ta - IL[0] - IR[0], tb - IL[-1] - IR[-1]])
    A, B = np.linalg.solve(mat, rhs)
    return IL + IR + A * ea + B * eb


def linv_periodic_direct(v, h, alpha, tol=1e-18):
    """L^{-1} v on a periodic line of n nodes (spacing h): direct sum over
    enough periodic images of every cell."""
    v = np.asarray(v, dtype=np.float64)
    n = len(v)
    L = n * h
    R = int(np.ceil(np.log(1.0 / tol) / (alpha * L))) + 1
    # extended node set covering the images -R..R plus one guard node each side
    k = np.arange(-R * n - 1, (R + 1) * n + 1)
    xe = k * h
    ve = v[k % n]
    out = np.zeros(n)
    for j in range(n):
        xj = j * h
        jj = j + R * n + 1           # index of x_j in the extended arrays
        s = 0.0
        for i in range(1, len(xe) - 1):
            if i <= jj:              # cell [x_{i-1}, x_i], interpolant of node i
                a, b = xe[i - 1], xe[i]
                kern = lambda y: 0.5 * alpha * np.exp(-alpha * (xj - y))  # noqa: E731
            else:
                continue
            xa, xb, xc = xe[i - 1], xe[i], xe[i + 1]
            va, vb, vc = ve[i - 1], ve[i], ve[i + 1]
            q = (lambda xa, xb, xc, va, vb, vc: lambda y: (
                va * (y - xb) * (y - xc) / ((xa - xb) * (xa - xc))
                + vb * (y - xa) * (y - xc) / ((xb - xa) * (xb - xc))
                + vc * (y - xa) * (y - xb) / ((xc - xa) * (xc - xb))))(xa, xb, xc, va, vb, vc)
            s += _cell_integral(lambda y: kern(y) * q(y), a, b, alpha)
        for i in range(1, len(xe) - 1):
            if i >= jj:              # cell [x_i, x_{i+1}], interpolant of node i
                a, b = xe[i], xe[i + 1]
                xa, xb, xc = xe[i - 1], xe[i], xe[i + 1]
                va, vb, vc = ve[i - 1], ve[i], ve[i + 1]
                q = (lambda xa, xb, xc, va, vb, vc: lambda y: (
                    va * (y - xb) * (y - xc) / ((xa - xb) * (xa - xc))
                    + vb * (y - xa) * (y - xc) / ((xb - xa) * (xb - xc))
                    + vc * (y - xa) * (y - xb) / ((xc - xa) * (xc - xb))))(xa, xb, xc, va, vb, vc)
                s += _cell_integral(lambda y: 0.5 * alpha * np.exp(-alpha * (y - xj)) * q(y),
                                    a, b, alpha)
        out[j] = s
    return out
