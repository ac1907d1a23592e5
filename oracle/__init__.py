"""Plain FP64 CPU oracle of the MOL^T recursive-convolution wave solver.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The HIP library
never does, and nothing here imports the HIP library.

Contents
--------
* ``molt_oracle.c`` (ctypes, FP64): O1 -- L^{-1} on a line by the two
  exponential recurrences plus the boundary correction (Sec. 2); the
  directional and ADI operators (Sec. 4, eqs. LD_gam, C_def_ADI(_3),
  D_def_ADI(_3)); the order-2P update with the Table 2 schedule; the
  three-level time step and the start step (Sec. 3.2).
* ``direct.py``: O2 -- the same discrete convolution evaluated directly as an
  O(M^2) Gauss-Legendre quadrature of the Green's function (eq. L_Inverse),
  with no recurrence and no closed-form weights.
* ``scheme.py``: A_p(beta) (Sec. 3, the A_p equation), c_{p,m} (eq. Full_2D),
  beta_max(P) (Theorem of Sec. 3.1, eq. Stab_cond).
* ``lines.py``: line objects of an embedded boundary (Sec. 4.3).
* ``Problem.step_source``: the step with a source term (Sec. 4, inclusion of
  source terms), P = 1 and 2, composed from the oracle's own step and C.
* ``Problem.start_g``: u^1 with an initial velocity (Sec. 3.2), the odd
  Taylor terms through the same schedule with the weights b_{p,m}.
* ``Problem.D_avg``, ``rhs_with``, ``step_avg``: D averaged over both orders of
  the directional inverses (Sec. 4, operation count: averaging the sweep
  permutations against the anisotropy) and the Table 2 schedule with a given
  D, in plain Python over the oracle's own L_gamma^{-1} and C.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import scheme  # noqa: F401  (re-export)
from .scheme import stage_coefficients, beta_max, A_p  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "molt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_LD = os.path.join(_HERE, "liboracle_ld.so")

DIRICHLET = 0
PERIODIC = 1


def build(force: bool = False) -> str:
    """Compile molt_oracle.c with gcc (-O2, OpenMP over lines): the FP64 oracle,
    and the same source with 80-bit long double arithmetic (long-run reference)."""
    for out, extra in ((_LIB, []), (_LIB_LD, ["-DOR_LONG_DOUBLE"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            tmp = out + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                                   *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, out)
    return _LIB


_libs = {}


def lib(precision: str = "f64"):
    """The oracle library: precision "f64" (double) or "ld" (x87 long double)."""
    if precision not in _libs:
        build()
        L = ctypes.CDLL(_LIB if precision == "f64" else _LIB_LD)
        rt = ctypes.c_double if precision == "f64" else ctypes.c_longdouble
        dp = ctypes.POINTER(rt)
        L.or_linv_line.argtypes = [ctypes.c_long, dp, dp, rt, dp, dp]
        L.or_linv_periodic_line.argtypes = [ctypes.c_long, rt, dp, rt, dp]
        for name in ("or_apply_C", "or_apply_D"):
            getattr(L, name).argtypes = [ctypes.c_void_p, dp, dp]
        for name in ("or_apply_linv", "or_apply_Dg"):
            getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
        L.or_rhs.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, dp]
        L.or_step.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, dp, dp]
        L.or_start.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, dp]
        L.or_run.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, dp, ctypes.c_long]
        L.or_num_threads.restype = ctypes.c_int
        L.or_count_get.restype = ctypes.c_long
        _libs[precision] = L
    return _libs[precision]


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    if a.dtype == np.float64:
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert a.dtype == np.longdouble
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_longdouble))


def _check(rc: int) -> None:
    if rc != 0:
        raise RuntimeError("oracle call failed with status %d" % rc)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_long * 3),
        ("h", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 3),
        ("alpha", ctypes.c_double),
        ("nseg", ctypes.c_long * 3),
        ("seg_idx", ctypes.c_void_p * 3),
        ("seg_th", ctypes.c_void_p * 3),
        ("mask", ctypes.c_void_p),
    ]


class Problem:
    """A grid problem: shape (C-order, x fastest), spacing, boundary types and
    alpha = beta/(c dt) (Sec. 2, eq. L_def).  ``segments`` = per-axis
    (seg_idx[n,3] int64, seg_th[n,2] float64) for embedded line objects
    (2D only), ``mask`` = uint8 inside indicator in the field's shape."""

    def __init__(self, shape, h, bc, alpha, segments=None, mask=None, precision="f64"):
        self.precision = precision
        self.rt = np.float64 if precision == "f64" else np.longdouble
        shape = tuple(int(s) for s in shape)
        self.shape = shape
        self.ndim = len(shape)
        nx = list(reversed(shape))  # n[0] = x (fastest)
        hh = list(h) if np.ndim(h) else [float(h)] * self.ndim
        bb = list(bc) if np.ndim(bc) else [int(bc)] * self.ndim
        s = _Problem()
        s.ndim = self.ndim
        for d in range(3):
            s.n[d] = nx[d] if d < self.ndim else 1
            s.h[d] = float(hh[d]) if d < self.ndim else 1.0
            s.bc[d] = int(bb[d]) if d < self.ndim else 0
        s.alpha = float(alpha)
        self._keep = []
        if segments is not None:
            for d, seg in enumerate(segments):
                if seg is None:
                    continue
                idx = np.ascontiguousarray(seg[0], dtype=np.int64)
                th = np.ascontiguousarray(seg[1], dtype=np.float64)
                self._keep += [idx, th]
                s.nseg[d] = idx.shape[0]
                s.seg_idx[d] = idx.ctypes.data
                s.seg_th[d] = th.ctypes.data
        self._mask = None
        if mask is not None:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            assert m.shape == shape
            self._keep.append(m)
            s.mask = m.ctypes.data
            self._mask = m.astype(np.float64)
        self._s = s
        self.alpha = float(alpha)

    @property
    def ref(self):
        return ctypes.byref(self._s)

    def _io(self, v):
        v = np.ascontiguousarray(v, dtype=self.rt)
        assert v.shape == self.shape, (v.shape, self.shape)
        return v, np.empty_like(v)

    def _lib(self):
        return lib(self.precision)

    def _coef(self, P, beta):
        if self.precision == "f64":
            return np.ascontiguousarray(stage_coefficients(P, beta), dtype=np.float64)
        return np.ascontiguousarray(scheme.stage_coefficients_ld(P, beta))

    @staticmethod
    def _out(a):
        return np.asarray(a, dtype=np.float64)

    def linv(self, v, axis):
        """L_gamma^{-1} along grid axis ``axis`` (0 = x, 1 = y, 2 = z)."""
        v, out = self._io(v)
        _check(self._lib().or_apply_linv(self.ref, axis, _p(v), _p(out)))
        return self._out(out)

    def Dg(self, v, axis):
        """D_gamma = 1 - L_gamma^{-1} (eq. LD_gam)."""
        v, out = self._io(v)
        _check(self._lib().or_apply_Dg(self.ref, axis, _p(v), _p(out)))
        return self._out(out)

    def C(self, v):
        v, out = self._io(v)
        _check(self._lib().or_apply_C(self.ref, _p(v), _p(out)))
        return self._out(out)

    def D(self, v):
        v, out = self._io(v)
        _check(self._lib().or_apply_D(self.ref, _p(v), _p(out)))
        return self._out(out)

    def rhs(self, u, P, beta):
        u, out = self._io(u)
        c = self._coef(P, beta)
        _check(self._lib().or_rhs(self.ref, P, _p(c), _p(u), _p(out)))
        return self._out(out)

    def step(self, u_prev, u_curr, P, beta):
        u_prev, _ = self._io(u_prev)
        u_curr, out = self._io(u_curr)
        c = self._coef(P, beta)
        _check(self._lib().or_step(self.ref, P, _p(c), _p(u_prev), _p(u_curr), _p(out)))
        return self._out(out)

    def source_terms(self, s_prev, s_curr, s_next, P, beta):
        """Source part of one step for u_tt / c^2 = laplacian(u) + S (Sec. 4,
        inclusion of source terms), with (c dt)^2 = (beta / alpha)^2.

        P = 1: (c dt)^2 S^n, the source part of the dt^2 term of the even
        Taylor series of u^{n+1} - 2 u^n + u^{n-1}.
        P = 2: (c dt)^2 / 12 (S^{n+1} + 10 S^n + S^{n-1})
               - beta^2 (c dt)^2 / 12 C[S^n].
        The second term is the dt^4 / 12 c^4 laplacian(S) term of the expansion
        with the laplacian replaced by -alpha^2 C, as the convolution operators
        replace it in the homogeneous part.  (The printed coefficient of
        C[S^n] has the dimension of the first term times a length^2; with it
        the scheme is second-order.)  FP64; s_prev and s_next are unused for
        P = 1."""
        if P not in (1, 2):
            raise ValueError("source terms are given for P = 1 and 2")
        a2 = (float(beta) / self.alpha) ** 2
        s_curr = np.asarray(s_curr, dtype=np.float64)
        if P == 1:
            return a2 * s_curr
        s_prev = np.asarray(s_prev, dtype=np.float64)
        s_next = np.asarray(s_next, dtype=np.float64)
        sig = a2 / 12.0
        return sig * (s_next + 10.0 * s_curr + s_prev) - float(beta) ** 2 * sig * self.C(s_curr)

    def step_source(self, u_prev, u_curr, s_prev, s_curr, s_next, P, beta):
        """u^{n+1} = 2 u^n - u^{n-1} + rhs(u^n) + source_terms (P = 1, 2), and
        u^{n+1} = 0 on the nodes of a Dirichlet boundary (homogeneous data,
        Sec. 2), as the homogeneous step gives there whatever S is."""
        out = self.step(u_prev, u_curr, P, beta) + self.source_terms(s_prev, s_curr, s_next, P, beta)
        return self._project_field(out)

    def _project_field(self, out):
        """A field of the solution: 0 on Dirichlet boundary nodes (homogeneous
        data) and on outside nodes of a mask."""
        out = np.array(out, dtype=np.float64)
        for d in range(self.ndim):
            if self._s.bc[d] == 0:
                ax = self.ndim - 1 - d          # grid axis d (x = 0) is array axis ndim-1-d
                idx = [slice(None)] * self.ndim
                idx[ax] = 0
                out[tuple(idx)] = 0.0
                idx[ax] = -1
                out[tuple(idx)] = 0.0
        return self._proj(out)

    def rhs_coef(self, u, coef):
        """The Table 2 schedule of the oracle's rhs with a given P x P weight
        matrix coef[p-1, m-1]."""
        u, out = self._io(u)
        c = np.ascontiguousarray(coef, dtype=self.rt)
        _check(self._lib().or_rhs(self.ref, c.shape[0], _p(c), _p(u), _p(out)))
        return self._out(out)

    def start_g(self, u0, g, P, beta, c=1.0):
        """u^1 with an initial velocity g (Sec. 3.2): the even Taylor terms
        u0 + rhs(u0)/2 and the odd ones dt (g + sum_{p<=P} sum_m b_{p,m}
        C^{m-1} D^{p-m} C g), dt = beta / (alpha c)."""
        dt = float(beta) / (self.alpha * c)
        g = np.asarray(g, dtype=np.float64)
        odd = dt * (g + self.rhs_coef(g, scheme.start_coefficients(P, beta)))
        return self._project_field(self.start(u0, P, beta) + odd)

    def _proj(self, v):
        """Zero outside nodes of a mask (they read and are written as 0)."""
        v = np.asarray(v, dtype=np.float64)
        return v * self._mask if self._mask is not None else v

    def D_avg(self, v):
        """v - (L_x^{-1} L_y^{-1} v + L_y^{-1} L_x^{-1} v) / 2 (2D): the D of
        eq. D_def_ADI averaged over the two orders of the inverses."""
        if self.ndim != 2:
            raise ValueError("the averaged D is defined here for 2D grids")
        v = self._proj(v)
        xy = self.linv(self.linv(v, 1), 0)
        yx = self.linv(self.linv(v, 0), 1)
        return self._proj(v - 0.5 * (self._proj(xy) + self._proj(yx)))

    def rhs_with(self, u, P, beta, D):
        """sum_p sum_m c_{p,m} C^{m-1} D^{p-m} C u in the order of Table 2
        (stage p: C on every earlier term, D on the newest one), with the
        operator D given; C is the oracle's."""
        c = stage_coefficients(P, beta)
        v = [self.C(self._proj(u))]
        out = c[0, 0] * v[0]
        for p in range(2, P + 1):
            v = [self.C(x) for x in v] + [D(v[-1])]
            for k, x in enumerate(v):            # term k carries p - k factors of C
                out = out + c[p - 1, p - k - 1] * x
        return self._proj(out)

    def step_avg(self, u_prev, u_curr, P, beta):
        """u^{n+1} = 2 u^n - u^{n-1} + rhs with the averaged D."""
        return self._proj(2.0 * np.asarray(u_curr, dtype=np.float64) - np.asarray(u_prev, dtype=np.float64)
                          + self.rhs_with(u_curr, P, beta, self.D_avg))

    def start(self, u0, P, beta):
        u0, out = self._io(u0)
        c = self._coef(P, beta)
        _check(self._lib().or_start(self.ref, P, _p(c), _p(u0), _p(out)))
        return self._out(out)

    def run(self, u_prev, u_curr, nsteps, P, beta):
        """Returns (u^{n+nsteps-1}, u^{n+nsteps})."""
        a = np.array(u_prev, dtype=self.rt, order="C", copy=True)
        b = np.array(u_curr, dtype=self.rt, order="C", copy=True)
        assert a.shape == self.shape and b.shape == self.shape
        c = self._coef(P, beta)
        _check(self._lib().or_run(self.ref, P, _p(c), _p(a), _p(b), int(nsteps)))
        return self._out(a), self._out(b)


def linv_line(x, v, alpha, bnd=None):
    """O1 on one bounded line object (nodes x, values v); bnd = (ta, tb, ka, kb)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty_like(v)
    b = np.ascontiguousarray(bnd if bnd is not None else (0.0, 0.0, 0.0, 0.0), dtype=np.float64)
    _check(lib("f64").or_linv_line(len(x) - 1, _p(x), _p(v), float(alpha), _p(b), _p(w)))
    return w


def linv_periodic_line(v, h, alpha):
    v = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty_like(v)
    _check(lib("f64").or_linv_periodic_line(len(v), float(h), _p(v), float(alpha), _p(w)))
    return w


def count_reset() -> None:
    """Reset the count of C/D operator applications (Table 2 pin)."""
    lib().or_count_reset()


def count_get() -> int:
    return int(lib().or_count_get())


def num_threads() -> int:
    return int(lib().or_num_threads())
