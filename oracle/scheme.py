"""Scheme coefficients of the order-2P family (test infrastructure; see the
package docstring).

* ``A_p(p, beta)``: A_p(beta) = 2 sum_{m=1}^{p} (-1)^m beta^{2m}/(2m)! binom(p-1, m-1)
  (Sec. 3, the A_p equation following eq. update_P).
* ``stage_coefficients(P, beta)``: c_{p,m} = (-1)^m 2 beta^{2m}/(2m)! binom(p-1, m-1),
  the weight of C^m D^{p-m} in eq. Full_2D (Sec. 4); sum_m c_{p,m} = A_p.
* ``start_coefficients(P, beta)``: b_{p,m} of the odd part of the start
  (Sec. 3.2 with the operator expansion of Sec. 4).
* ``beta_max(P)``: the first positive root of -sum_{p<=P} A_p(beta) = 4
  (Theorem of Sec. 3.1, eq. Stab_cond), i.e. S(beta, 1) = 4 with S from
  eq. Stab_sum.
"""
from __future__ import annotations

from fractions import Fraction
from math import comb, factorial

import mpmath as mp
import numpy as np


def A_poly(p: int):
    """Exact rational coefficients a_m of A_p(beta) = sum_m a_m beta^{2m}."""
    return [Fraction(2 * (-1) ** m * comb(p - 1, m - 1), factorial(2 * m)) for m in range(1, p + 1)]


def A_p(p: int, beta):
    """A_p(beta); exact when beta is a Fraction, else evaluated in its type."""
    return sum(a * beta ** (2 * m) for m, a in enumerate(A_poly(p), start=1))


def c_pm(p: int, m: int, beta):
    return Fraction(2 * (-1) ** m * comb(p - 1, m - 1), factorial(2 * m)) * beta ** (2 * m) \
        if isinstance(beta, Fraction) else \
        2.0 * (-1) ** m * comb(p - 1, m - 1) / factorial(2 * m) * float(beta) ** (2 * m)


def b_pm(p: int, m: int, beta):
    """Weight of C^m D^{p-m} in the odd part of the start (Sec. 3.2): the
    series sum_m beta^{2m}/(2m+1)! (laplacian/alpha^2)^m with
    (laplacian/alpha^2)^m = (-1)^m C^m (1 - D)^{-m} (the expansion behind
    eq. Full_2D): b_{p,m} = (-1)^m beta^{2m}/(2m+1)! binom(p-1, m-1)."""
    if isinstance(beta, Fraction):
        return Fraction((-1) ** m * comb(p - 1, m - 1), factorial(2 * m + 1)) * beta ** (2 * m)
    return (-1) ** m * comb(p - 1, m - 1) / factorial(2 * m + 1) * float(beta) ** (2 * m)


def start_coefficients(P: int, beta: float) -> np.ndarray:
    """P x P matrix, entry [p-1, m-1] = b_{p,m} (zero for m > p)."""
    c = np.zeros((P, P), dtype=np.float64)
    for p in range(1, P + 1):
        for m in range(1, p + 1):
            c[p - 1, m - 1] = b_pm(p, m, beta)
    return c


def stage_coefficients(P: int, beta: float) -> np.ndarray:
    """P x P matrix, entry [p-1, m-1] = c_{p,m} (zero for m > p)."""
    c = np.zeros((P, P), dtype=np.float64)
    for p in range(1, P + 1):
        for m in range(1, p + 1):
            c[p - 1, m - 1] = c_pm(p, m, beta)
    return c


def stage_coefficients_ld(P: int, beta: float) -> np.ndarray:
    """c_{p,m} in extended precision (numpy longdouble) for the 80-bit build;
    beta is taken as the exact binary value of the given double."""
    c = np.zeros((P, P), dtype=np.longdouble)
    b = Fraction(float(beta))
    for p in range(1, P + 1):
        for m in range(1, p + 1):
            q = c_pm(p, m, b)
            with mp.workdps(40):
                c[p - 1, m - 1] = np.longdouble(mp.nstr(mp.mpf(q.numerator) / q.denominator, 30))
    return c


def stability_S(P: int, beta, Dhat):
    """S(beta, Dhat) = -sum_{p<=P} A_p(beta) Dhat^p (eq. Stab_sum)."""
    return -sum(A_p(p, beta) * Dhat ** p for p in range(1, P + 1))


def beta_max(P: int, dps: int = 30) -> float:
    """First positive root of S(beta, 1) = 4, found by a fine scan from beta = 0
    followed by bisection, in ``dps`` decimal digits."""
    with mp.workdps(dps):
        f = lambda b: stability_S(P, mp.mpf(b), 1) - 4  # noqa: E731
        step = mp.mpf("0.001")
        b = step
        while f(b) < 0:
            b += step
            if b > 10:
                raise RuntimeError("no root below 10")
        lo, hi = b - step, b
        for _ in range(200):
            mid = (lo + hi) / 2
            if f(mid) < 0:
                lo = mid
            else:
                hi = mid
        return float((lo + hi) / 2)
