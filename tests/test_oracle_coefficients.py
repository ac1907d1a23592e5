"""Pins of the scheme coefficients: Table 1, the explicit updates of Sec. 3 and
Sec. 4, the stability sum, and the untruncated series."""
from fractions import Fraction

import mpmath as mp
import pytest

from conftest import golden
from oracle import scheme


def test_explicit_updates_sec3():
    # eqs. update_1..update_3: A_1 = -b^2, A_2 = -(b^2 - b^4/12),
    # A_3 = -(b^2 - b^4/6 + b^6/360)
    for b in (Fraction(1), Fraction(3, 2), Fraction(7, 5), Fraction(2)):
        b2 = b * b
        assert scheme.A_p(1, b) == -b2
        assert scheme.A_p(2, b) == -(b2 - b2 * b2 / 12)
        assert scheme.A_p(3, b) == -(b2 - b2 * b2 / 6 + b2 ** 3 / 360)


def test_explicit_adi_truncations_sec4():
    # printed P = 2, 3 truncations of eq. Full_2D:
    #   -b^2 C - (b^2 D - b^4/12 C) C - (b^2 D^2 - b^4/6 C D + b^6/360 C^2) C
    b = Fraction(13, 10)
    b2 = b * b
    assert scheme.c_pm(1, 1, b) == -b2
    assert scheme.c_pm(2, 1, b) == -b2          # D C
    assert scheme.c_pm(2, 2, b) == b2 * b2 / 12  # C C
    assert scheme.c_pm(3, 1, b) == -b2          # D D C
    assert scheme.c_pm(3, 2, b) == b2 * b2 / 6   # C D C
    assert scheme.c_pm(3, 3, b) == -b2 ** 3 / 360


@pytest.mark.parametrize("p", range(1, 8))
def test_setting_C_equal_D_recovers_1d(p):
    # Sec. 4: the 1D scheme is the case C = D, so sum_m c_{p,m} = A_p
    b = Fraction(6, 5)
    assert sum(scheme.c_pm(p, m, b) for m in range(1, p + 1)) == scheme.A_p(p, b)


def test_untruncated_series_is_the_taylor_expansion():
    # eq. exact + the D-expansion: sum_p A_p Dh^p = 2 (cos(b k/alpha) - 1) with
    # (k/alpha)^2 = Dh / (1 - Dh); converges for Dh < 1.
    with mp.workdps(30):
        for b in (mp.mpf("0.7"), mp.mpf("1.3")):
            for Dh in (mp.mpf("0.05"), mp.mpf("0.3")):
                s = sum(scheme.A_p(p, b) * Dh ** p for p in range(1, 120))
                exact = 2 * (mp.cos(b * mp.sqrt(Dh / (1 - Dh))) - 1)
                assert abs(s - exact) < mp.mpf("1e-25")


def test_table1_beta_max():
    rows = golden("table1_beta_max.txt")
    for P_s, order_s, printed_s in rows:
        P, printed = int(P_s), float(printed_s)
        assert int(order_s) == 2 * P
        b = scheme.beta_max(P)
        # the root satisfies S(beta_max, 1) = 4 (eq. Stab_cond)
        assert abs(float(scheme.stability_S(P, mp.mpf(b), 1)) - 4.0) < 1e-12
        if P == 3:
            # printed 1.2345; the root is 1.234291 (a rounding slip in the table):
            # at the printed value S(beta, 1) exceeds 4, i.e. it is not stable.
            assert abs(b - 1.234291) < 1e-6
            assert float(scheme.stability_S(3, mp.mpf(printed), 1)) > 4.0
        else:
            # within one unit of the last printed digit (P = 2 prints 1.4840 for
            # the root 1.483928)
            assert abs(b - printed) <= 1e-4


@pytest.mark.parametrize("P", range(1, 6))
def test_stability_range(P):
    # for 0 < beta <= beta_max and 0 <= Dhat <= 1: 0 <= S <= 4 (Cohn-Schur, Sec. 3.1)
    # and every A_p < 0 (the Lemma of Sec. 3.1)
    bm = scheme.beta_max(P)
    for i in range(1, 21):
        b = bm * i / 20
        for p in range(1, P + 1):
            assert scheme.A_p(p, b) < 0
        for j in range(0, 21):
            S = scheme.stability_S(P, b, j / 20)
            assert -1e-14 <= S <= 4 + 1e-12
    # just above beta_max the bound fails at Dhat = 1
    assert scheme.stability_S(P, bm * 1.001, 1.0) > 4
