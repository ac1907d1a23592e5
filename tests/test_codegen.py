"""Code-generation check of the chained strided sweep (CPU only: hipcc
cross-compiles gfx950).  The kernel keeps its loads two sub-tiles ahead of
their use; a load issued under a branch makes the compiler wait for every load
in flight where the branch rejoins (`s_waitcnt vmcnt(0)`), which serialises the
prefetch and cost 10 % of the kernel's time when it happened.  The default
configuration, plain and batched entry points, must contain no such wait."""
import os
import re
import shutil
import subprocess

import pytest

from conftest import ROOT

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SRC = os.path.join(ROOT, "paper_1308_3214_amd", "csrc", "molt_sweep_yy32.hip")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("cg") / "yy.s")
    from paper_1308_3214_amd import build
    cmd = [HIPCC, *[f for f in build.FLAGS if f != "-fPIC"], "--cuda-device-only", "-S", "-x", "hip",
           SRC, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


def _body(asm, pattern):
    names = [n for n in re.findall(r"^(_ZN4molt\w+):", asm, re.M) if re.search(pattern, n)]
    assert names, pattern
    out = {}
    for n in names:
        i = asm.index(n + ":")
        out[n] = asm[i:asm.index(".Lfunc_end", i)]
    return out


def test_chained_sweep_prefetch_not_serialised(asm):
    # k_sweep_yy<float, S=8, W=8, NO=2, Dirichlet and periodic, NFP=3>, plain and batched
    bodies = _body(asm, r"k_sweep_yy(_b)?IfLi8ELi8ELi2ELb[01]ELi3E")
    assert len(bodies) == 4
    bad = []
    for name, body in bodies.items():
        waits = re.findall(r"s_waitcnt vmcnt\(0\)", body)
        loads = re.findall(r"buffer_load_dword", body)
        print(name, "loads", len(loads), "full waits", len(waits))
        assert len(loads) > 0
        if waits:
            bad.append(name)
    assert not bad, bad
