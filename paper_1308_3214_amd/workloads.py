"""Seeded synthetic inputs for the wave solver.

This module holds only input generation: grids, initial data, masks and
boundary crossings, request streams.  It contains none of the solver's
arithmetic, and both the HIP path and the CPU oracle draw their inputs from it.
Everything is generated on the host in FP64 with NumPy's PCG64 generator.

Conventions (c = 1):
* Dirichlet unit interval / square / cube: n nodes per axis at j/(n-1),
  boundary nodes included (h = 1/(n-1)); boundary values are 0.
* Periodic unit cube: n nodes per axis at j/n.
* dt = CFL * h; the scheme parameter alpha = beta/dt and nu = alpha h = beta/CFL.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# 1D standing modes
# --------------------------------------------------------------------------
def sine_modes_1d(n: int = 1024, seed: int = 1, modes=(1, 3)):
    """u0 = sum_k a_k sin(k pi x) on [0, 1], a_k ~ U[0.5, 1]; returns (x, u0, amplitudes)."""
    g = rng(seed)
    x = np.arange(n, dtype=np.float64) / (n - 1)
    amps = g.uniform(0.5, 1.0, size=len(modes))
    u = np.zeros(n)
    for a, k in zip(amps, modes):
        u += a * np.sin(k * np.pi * x)
    u[0] = u[-1] = 0.0
    return x, u, amps


# --------------------------------------------------------------------------
# 2D Gaussian pulses on the unit square
# --------------------------------------------------------------------------
def gaussian_pulses_2d(n: int, seed: int = 1, npulses: int = 8, sigma: float = 0.02,
                       lo: float = 0.2, hi: float = 0.8, ny: int | None = None):
    """Sum of pulses A_i exp(-|x - c_i|^2 / (2 sigma^2)), c_i ~ U[lo, hi]^2,
    A_i ~ U[0.5, 1], on an (ny, n) Dirichlet grid of the unit square; the
    boundary ring is set to 0.  Returns the (ny, n) field."""
    ny = n if ny is None else ny
    g = rng(seed)
    cen = g.uniform(lo, hi, size=(npulses, 2))
    amp = g.uniform(0.5, 1.0, size=npulses)
    x = np.arange(n, dtype=np.float64) / (n - 1)
    y = np.arange(ny, dtype=np.float64) / (ny - 1)
    u = np.zeros((ny, n))
    for (cx, cy), a in zip(cen, amp):
        gx = np.exp(-(x - cx) ** 2 / (2 * sigma * sigma))
        gy = np.exp(-(y - cy) ** 2 / (2 * sigma * sigma))
        u += a * np.outer(gy, gx)
    u[0, :] = u[-1, :] = 0.0
    u[:, 0] = u[:, -1] = 0.0
    return u


def random_field(shape, seed: int = 1, dirichlet_axes=()):
    """Uniform random data in [-1, 1] (kernel parity tests); zero on the
    boundary nodes of the listed axes (0 = x, the last array axis)."""
    g = rng(seed)
    u = g.uniform(-1.0, 1.0, size=shape)
    nd = len(shape)
    for ax in dirichlet_axes:
        arr_ax = nd - 1 - ax
        sl = [slice(None)] * nd
        sl[arr_ax] = 0
        u[tuple(sl)] = 0.0
        sl[arr_ax] = -1
        u[tuple(sl)] = 0.0
    return u


def table3_mode(n: int = 641):
    """sin(pi x) sin(pi y) on [-1, 1]^2 with n x n nodes (the refinement study of
    the ADI section); returns (field, h)."""
    x = -1.0 + 2.0 * np.arange(n, dtype=np.float64) / (n - 1)
    s = np.sin(np.pi * x)
    s[0] = s[-1] = 0.0
    return np.outer(s, s), 2.0 / (n - 1)


def sine_mode(n: int, ndim: int):
    """prod_k sin(pi x_k) on [-1, 1]^ndim with n nodes per direction (zero on
    the boundary nodes); returns (field, h)."""
    x = -1.0 + 2.0 * np.arange(n, dtype=np.float64) / (n - 1)
    s = np.sin(np.pi * x)
    s[0] = s[-1] = 0.0
    f = s
    for _ in range(ndim - 1):
        f = np.multiply.outer(s, f)
    return np.ascontiguousarray(f), 2.0 / (n - 1)


def point_source_fig3(n: int = 81, periods_per_unit: float = 1.0, ramp: float = 0.3):
    """The point-source run of the ADI section's figure (80 x 80 cells on
    [-1, 1]^2, CFL 2): a discrete delta at the centre node (G = 1/h^2 there)
    and the signal f(t) = sin(2 pi k t) (1 - exp(-(t / ramp)^2)), switched on
    smoothly from f = 0 at t = 0 (frequency and ramp are not stated; k = 1 and
    ramp 0.3 resolve a period in 20 steps).  Returns (G, f, h)."""
    h = 2.0 / (n - 1)
    G = np.zeros((n, n))
    G[n // 2, n // 2] = 1.0 / h ** 2

    def f(t):
        t = np.asarray(t, dtype=np.float64)
        return np.where(t > 0, np.sin(2 * np.pi * periods_per_unit * t) * (1 - np.exp(-(t / ramp) ** 2)), 0.0)
    return G, f, h


# --------------------------------------------------------------------------
# 3D plane waves on the periodic unit cube
# --------------------------------------------------------------------------
def plane_waves_3d(n: int = 256, seed: int = 1, nwaves: int = 4, kmax: float = 16.0):
    """u0 = sum_i (1/4) cos(2 pi k_i . x + phi_i), k_i in Z^3 \\ {0}, |k_i| <= kmax,
    phi_i ~ U[0, 2 pi), on n^3 nodes x = j/n.  Returns (field (n,n,n) [z,y,x],
    wavevectors (nwaves, 3) as (kx, ky, kz), phases)."""
    g = rng(seed)
    ks = []
    kk = int(np.floor(kmax))
    while len(ks) < nwaves:
        k = g.integers(-kk, kk + 1, size=3)
        if 0 < np.dot(k, k) <= kmax * kmax:
            ks.append(k)
    ks = np.array(ks, dtype=np.int64)
    ph = g.uniform(0.0, 2 * np.pi, size=nwaves)
    x = np.arange(n, dtype=np.float64) / n
    u = np.zeros((n, n, n))
    for (kx, ky, kz), p in zip(ks, ph):
        u += 0.25 * np.cos(2 * np.pi * (kx * x[None, None, :] + ky * x[None, :, None]
                                        + kz * x[:, None, None]) + p)
    return u, ks, ph


# --------------------------------------------------------------------------
# Star-shaped cavity with an embedded boundary
# --------------------------------------------------------------------------
@dataclass
class StarDomain:
    n: int
    a: np.ndarray            # a_1..a_6
    center: tuple = (0.5, 0.5)
    base: float = 0.4
    amp: float = 0.2

    def radius(self, theta):
        k = np.arange(1, len(self.a) + 1)
        return self.base * (1.0 + self.amp * np.cos(np.multiply.outer(theta, k)) @ self.a)

    def inside(self, px, py):
        dx, dy = px - self.center[0], py - self.center[1]
        return np.hypot(dx, dy) < self.radius(np.arctan2(dy, dx))


def star_domain(n: int = 2048, seed: int = 1):
    """Star-shaped domain r(theta) = 0.4 (1 + 0.2 sum_{k<=6} a_k cos(k theta)),
    a_k ~ U[-1, 1] rescaled to sum |a_k| = 1, centred in the unit square, on an
    n x n grid with h = 1/(n-1).  Returns (StarDomain, mask (n, n) uint8,
    cross (4, n, n) float64): cross[d] at an inside node next to an outside
    node is the distance to the boundary crossing in units of h toward -x, +x,
    -y, +y (found by bisection in FP64), NaN elsewhere."""
    g = rng(seed)
    a = g.uniform(-1.0, 1.0, size=6)
    a /= np.abs(a).sum()
    dom = StarDomain(n=n, a=a)
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)           # [y, x]
    mask = dom.inside(X, Y).astype(np.uint8)
    mask[0, :] = mask[-1, :] = 0
    mask[:, 0] = mask[:, -1] = 0
    cross = np.full((4, n, n), np.nan)
    dirs = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    for d, (sx, sy) in enumerate(dirs):
        nb = np.roll(mask, shift=(-sy, -sx), axis=(0, 1))
        jj, ii = np.nonzero((mask == 1) & (nb == 0))
        px, py = x[ii], x[jj]
        lo = np.zeros(len(ii))
        hi = np.ones(len(ii))
        for _ in range(60):            # bisection on the segment node -> neighbour
            mid = 0.5 * (lo + hi)
            ins = dom.inside(px + sx * mid * h, py + sy * mid * h)
            lo = np.where(ins, mid, lo)
            hi = np.where(ins, hi, mid)
        cross[d, jj, ii] = np.clip(0.5 * (lo + hi), 1e-12, 1.0)
    return dom, mask, cross


def star_pulses(dom: StarDomain, mask, seed: int = 1, npulses: int = 16, sigma: float = 0.02):
    """Initial pulses A_i exp(-|x - c_i|^2/(2 sigma^2)), A_i ~ U[0.5, 1], with
    centres drawn uniformly inside 0.7 r(theta); zero outside the domain."""
    g = rng(seed + 1000)
    n = dom.n
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    cen = []
    while len(cen) < npulses:
        th = g.uniform(0, 2 * np.pi)
        r = np.sqrt(g.uniform(0, 1)) * 0.7 * dom.radius(np.array([th]))[0]
        cen.append((dom.center[0] + r * np.cos(th), dom.center[1] + r * np.sin(th)))
    amp = g.uniform(0.5, 1.0, size=npulses)
    u = np.zeros((n, n))
    for (cx, cy), A in zip(cen, amp):
        u += A * np.outer(np.exp(-(x - cy) ** 2 / (2 * sigma ** 2)),
                          np.exp(-(x - cx) ** 2 / (2 * sigma ** 2)))
    u *= mask
    return u


def ellipse_domain(n: int = 256):
    """The elliptical cavity of the ADI section, ((x+y)/4)^2 + (x-y)^2 = 1,
    scaled into the unit square (x, y -> (X - 0.5) * 6, ...): returns (mask, cross)
    in the same layout as ``star_domain``."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h

    def inside(px, py):
        u, v = (px - 0.5) * 6.0, (py - 0.5) * 6.0
        return ((u + v) / 4.0) ** 2 + (u - v) ** 2 < 1.0
    X, Y = np.meshgrid(x, x)
    mask = inside(X, Y).astype(np.uint8)
    mask[0, :] = mask[-1, :] = 0
    mask[:, 0] = mask[:, -1] = 0
    cross = np.full((4, n, n), np.nan)
    for d, (sx, sy) in enumerate([(-1, 0), (1, 0), (0, -1), (0, 1)]):
        nb = np.roll(mask, shift=(-sy, -sx), axis=(0, 1))
        jj, ii = np.nonzero((mask == 1) & (nb == 0))
        px, py = x[ii], x[jj]
        lo, hi = np.zeros(len(ii)), np.ones(len(ii))
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            ins = inside(px + sx * mid * h, py + sy * mid * h)
            lo = np.where(ins, mid, lo)
            hi = np.where(ins, hi, mid)
        cross[d, jj, ii] = np.clip(0.5 * (lo + hi), 1e-12, 1.0)
    return mask, cross


# --------------------------------------------------------------------------
# Serving stream
# --------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    P: int
    cfl: float
    steps: int
    seed: int
    extra: dict = field(default_factory=dict)


def request_stream(count: int = 256, rate_hz: float = 50.0, seed: int = 1, steps: int = 100,
                   nmin: int = 128, nmax: int = 2048, burst: bool = False):
    """Poisson arrivals (exponential gaps, mean 1/rate), grid side
    round(nmin * (nmax/nmin)^U) (log-uniform), P ~ U{1,2,3}, CFL ~ U[1, 4]."""
    g = rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        if not burst:
            t += g.exponential(1.0 / rate_hz)
        n = int(round(nmin * (nmax / nmin) ** g.uniform()))
        P = int(g.integers(1, 4))
        cfl = float(g.uniform(1.0, 4.0))
        out.append(Request(rid=i, arrival_s=0.0 if burst else t, n=n, P=P, cfl=cfl,
                           steps=steps, seed=int(seed * 100003 + i)))
    return out


def request_initial(req: Request):
    return gaussian_pulses_2d(req.n, seed=req.seed, npulses=4)
