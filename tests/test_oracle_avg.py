"""Pins of the oracle's averaged D (Sec. 4, operation count: averaging the
permutations of the directional inverses against the anisotropy of ADI).

* The Python Table 2 schedule ``rhs_with`` given the oracle's literal D equals
  the oracle's own rhs (C source, pinned by Table 3 and the closed forms).
* On the ellipse of the ADI section, which is symmetric under x <-> y, the
  averaged D and every rhs built on it commute with transposition to rounding,
  while the literal D = 1 - L_x^{-1} L_y^{-1} does not (so an average that is
  not taken, or taken over one order twice, fails).
* On a rectangle (mask = whole interior) the two orders commute: the averaged
  D equals the literal one; P = 1 has no D and is unchanged.
"""
import numpy as np
import pytest

from oracle import lines, scheme
from paper_1308_3214_amd import workloads as W


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def ellipse(oracle_mod):
    mask, cross = W.ellipse_domain(64)
    h = 1.0 / 63
    assert np.array_equal(mask, mask.T)
    pb = oracle_mod.Problem(mask.shape, h, 0, scheme.beta_max(2) / (2 * h),
                            segments=lines.segments(mask, cross), mask=mask)
    v = W.random_field(mask.shape, seed=11) * mask
    return pb, v


def test_python_schedule_equals_the_oracle_rhs(ellipse, oracle_mod):
    pb, v = ellipse
    dom, mask, cross = W.star_domain(72, seed=2)
    ps = oracle_mod.Problem(mask.shape, 1.0 / 71, 0, 40.0, segments=lines.segments(mask, cross), mask=mask)
    vs = W.random_field(mask.shape, seed=12) * mask
    for P in (1, 2, 3):
        b = scheme.beta_max(P)
        for p_, x in ((pb, v), (ps, vs)):
            e = _rel(p_.rhs_with(x, P, b, p_.D), p_.rhs(x, P, b))
            assert e < 1e-14, (P, e)


def test_averaged_d_commutes_with_transposition(ellipse):
    pb, v = ellipse
    vt = np.ascontiguousarray(v.T)
    e_avg = _rel(pb.D_avg(vt), pb.D_avg(v).T)
    e_lit = _rel(pb.D(vt), pb.D(v).T)
    print("transposition defect: averaged D %.2e, literal D %.2e" % (e_avg, e_lit))
    assert e_avg < 1e-14
    assert e_lit > 1e-3
    for P in (2, 3):
        b = scheme.beta_max(P)
        e = _rel(pb.rhs_with(vt, P, b, pb.D_avg), pb.rhs_with(v, P, b, pb.D_avg).T)
        e_l = _rel(pb.rhs(vt, P, b), pb.rhs(v, P, b).T)
        print("P=%d rhs transposition defect: averaged %.2e, literal %.2e" % (P, e, e_l))
        assert e < 1e-14 and e_l > 1e-6


def test_averaged_d_on_a_rectangle_and_p1(ellipse, oracle_mod):
    ny, nx = 40, 52
    mask = np.zeros((ny, nx), np.uint8)
    mask[1:-1, 1:-1] = 1
    pb = oracle_mod.Problem(mask.shape, 1.0 / (nx - 1), 0, 30.0,
                            segments=lines.segments(mask, None), mask=mask)
    v = W.random_field(mask.shape, seed=13) * mask
    assert _rel(pb.D_avg(v), pb.D(v)) < 1e-13
    pe, ve = ellipse
    b = scheme.beta_max(1)
    assert _rel(pe.rhs_with(ve, 1, b, pe.D_avg), pe.rhs(ve, 1, b)) < 1e-15
