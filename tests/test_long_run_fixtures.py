"""Integrity of the sampled long-run oracle fixtures under tests/golden/
(written by tests/golden/make_long_runs.py): the parameters in each header
are the ones the oracle derives for the stated grid, order and CFL number
(beta_max(P) of the stability analysis, Sec. 3.1; alpha = beta / (CFL h)),
and the samples are well formed.  CPU only."""
import os
import re

import numpy as np
import pytest

from conftest import ROOT

import oracle

GOLDEN = os.path.join(ROOT, "tests", "golden")

# name: (n, P, CFL)
BOX = {
    "adi4096_p2_cfl2_10": (4096, 2, 2.0),
    "adi4096_p2_cfl10_10": (4096, 2, 10.0),
    "adi4096_p2_cfl100_10": (4096, 2, 100.0),
    "adi4096_p2_cfl1000_10": (4096, 2, 1000.0),
    "config2_1024_p2_cfl2_500": (1024, 2, 2.0),
    "star2048_p3_cfl15_20": (2048, 3, 1.5),
    "star512_p3_cfl15_300": (512, 3, 1.5),
}


def _load(name):
    head, l2, mx, idx, val = [], None, None, [], []
    with open(os.path.join(GOLDEN, name + ".txt")) as f:
        for line in f:
            if line.startswith("#"):
                head.append(line[1:].strip())
                continue
            a, b = line.split()
            if a == "l2norm":
                l2 = float(b)
            elif a == "maxabs":
                mx = float(b)
            else:
                idx.append(int(a))
                val.append(float(b))
    return head, l2, mx, np.array(idx), np.array(val)


@pytest.mark.parametrize("name", sorted(BOX))
def test_fixture_parameters_and_samples(name):
    n, P, cfl = BOX[name]
    head, l2, mx, idx, val = _load(name)
    # the header names the CFL number and order it was written for
    assert ("CFL %g" % cfl) in head[0] and ("P = %d" % P) in head[0], head[0]
    m = re.match(r"beta (\S+) alpha (\S+)", [h for h in head if h.startswith("beta ")][0])
    beta, alpha = float(m.group(1)), float(m.group(2))
    h = 1.0 / (n - 1)
    b_or = float(oracle.beta_max(P))
    assert abs(beta / b_or - 1.0) < 1e-14
    assert abs(alpha / (b_or / (cfl * h)) - 1.0) < 1e-14
    # samples: distinct in-range nodes, finite values within the stated max
    assert idx.size >= 1024 and np.unique(idx).size == idx.size
    assert idx.min() >= 0 and idx.max() < n * n
    assert np.isfinite(val).all() and np.isfinite(l2) and l2 > 0
    assert np.abs(val).max() <= mx * (1 + 1e-15)
    # box domains: the lines next to the boundary are sampled (rows 1 and
    # n-2, columns 1 and n-2), where line-end closures act (a star cavity
    # does not reach those lines)
    if not name.startswith("star"):
        r, c = idx // n, idx % n
        for sel in (r == 1, r == n - 2, c == 1, c == n - 2):
            assert sel.sum() >= 16
