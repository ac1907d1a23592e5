"""Build libmolt.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import fcntl
import hashlib
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmolt.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = (["molt_sweep_%s%s_n%d.hip" % (k, t, n) for k in ("x", "s") for t in ("32", "64")
            for n in (4, 16)]
           + ["molt_sweep_p%s_p%d.hip" % (t, n) for t in ("32", "64") for n in (1, 2, 4)]
           + ["molt_sweep_e%s_n%d.hip" % (t, n) for t in ("32", "64") for n in (4, 16)]
           + ["molt_sweep_yy32.hip", "molt_kernels.hip", "molt_plan.cpp", "molt_masked.cpp", "molt_seg.hip",
              "molt_server.cpp", "molt_static.hip"])
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # no packed-FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _includes(path: str, seen: set) -> None:
    """The library's own headers path includes, transitively (quoted
    includes resolved beside the including file)."""
    with open(path) as f:
        for line in f:
            m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
            if m:
                dep = os.path.normpath(os.path.join(os.path.dirname(path), m.group(1)))
                if dep not in seen and os.path.exists(dep):
                    seen.add(dep)
                    _includes(dep, seen)


def _inputs_digest(src: str) -> str:
    """Digest of what an object is compiled from: the source, the headers it
    includes (transitively) and the flags."""
    h = hashlib.sha256()
    h.update(" ".join(FLAGS).encode())
    path = os.path.join(CSRC, src)
    deps = set()
    _includes(path, deps)
    for dep in [path] + sorted(deps):
        with open(dep, "rb") as f:
            h.update(os.path.basename(dep).encode())
            h.update(f.read())
    return h.hexdigest()


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    stamp = obj + ".stamp"
    digest = _inputs_digest(src)
    if incremental and os.path.exists(obj) and os.path.exists(stamp):
        with open(stamp) as f:
            if f.read().strip() == digest:
                return obj
    if os.path.exists(stamp):
        os.remove(stamp)
    tmp = obj + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + src)
    os.replace(tmp, obj)
    # the digest was taken before the compile: a source changed meanwhile
    # leaves a stale stamp, and the next incremental build compiles again
    with open(stamp, "w") as f:
        f.write(digest + "\n")
    return obj


def build(jobs: int = 8, out: str = OUT, incremental: bool = False) -> str:
    """Compile every source (incremental: only those whose source, headers or
    flags differ from what their object was compiled from) and link the
    library.  One build at a time: a second one waits for the first, so that
    no object is compiled from one state of the headers and linked with
    objects of another."""
    os.makedirs(BUILD, exist_ok=True)
    with open(os.path.join(BUILD, ".lock"), "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            objs = list(ex.map(lambda s: _compile(s, incremental), srcs))
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-ldl"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("link failed")
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--incremental"]
    print(build(out=args[0] if args else OUT, incremental="--incremental" in sys.argv))
