"""Thin ctypes binding of libmolt.so (the C-ABI declared in include/molt.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  torch supplies device memory and streams.  If the shared library is
missing this module raises at import time; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MOLT_LIB") or os.path.join(_HERE, "libmolt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libmolt.so is not built (run __graft_entry__.build() or "
                      "python paper_1308_3214_amd/build.py)")

# torch (the binding's device memory and streams) loads first, so that the
# library binds to the HIP runtime torch already holds: with the library
# loaded first, torch's later device initialisation found no GPU
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIB_PATH)

# status codes / enums (include/molt.h)
MOL_OK, MOL_E_INVALID, MOL_E_UNSUPPORTED, MOL_E_UNSTABLE, MOL_E_NOMEM, MOL_E_DEVICE = range(6)
DIRICHLET, PERIODIC, NEUMANN = 0, 1, 2
F64, F32 = 0, 1
ALLOW_UNSTABLE, INCREMENT_FORM, NO_GRAPH, SPLIT_Y, UNIFORM_CONFIG, SYMMETRIC_D = 1, 2, 4, 8, 16, 32
OPS = {"linv_x": 0, "linv_y": 1, "linv_z": 2, "d_x": 3, "d_y": 4, "d_z": 5, "C": 6, "D": 7, "rhs": 8}
_STATUS = {1: "MOL_E_INVALID", 2: "MOL_E_UNSUPPORTED", 3: "MOL_E_UNSTABLE", 4: "MOL_E_NOMEM",
           5: "MOL_E_DEVICE"}


class MolError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int64 * 3),
        ("h", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 3),
        ("mask", ctypes.c_void_p),
        ("cross", ctypes.c_void_p),
        ("P", ctypes.c_int),
        ("c", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("dtype", ctypes.c_int),
        ("flags", ctypes.c_int),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("beta", ctypes.c_double),
        ("beta_max", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("nu", ctypes.c_double * 3),
        ("points", ctypes.c_int64),
        ("unknowns", ctypes.c_int64),
        ("segments", ctypes.c_int64 * 2),
        ("kernels_per_step", ctypes.c_int),
        ("bytes_per_step", ctypes.c_double),
        ("workspace_bytes", ctypes.c_size_t),
        ("kernels_per_source_step", ctypes.c_int),
        ("bytes_per_source_step", ctypes.c_double),
    ]


_vp = ctypes.c_void_p
_lib.mol_beta_max.argtypes = [ctypes.c_int]
_lib.mol_beta_max.restype = ctypes.c_double
_lib.mol_last_error.restype = ctypes.c_char_p
_lib.mol_workspace_bytes.argtypes = [ctypes.POINTER(_Desc)]
_lib.mol_workspace_bytes.restype = ctypes.c_size_t
_lib.mol_plan_create.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(_vp)]
_lib.mol_plan_destroy.argtypes = [_vp]
_lib.mol_plan_get_info.argtypes = [_vp, ctypes.POINTER(_Info)]
_lib.mol_start.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.mol_step.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.mol_step_source.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.mol_solve_source.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp]
_lib.mol_solve.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp]
_lib.mol_solve_prepare.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp]
_lib.mol_step_static.argtypes = [ctypes.POINTER(_Desc), _vp, _vp, _vp, _vp]
_lib.mol_step_bdata.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp]
_lib.mol_step_static_max_bytes.restype = ctypes.c_size_t
_lib.mol_apply.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
_lib.mol_step_batch.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                ctypes.POINTER(_vp), ctypes.c_int, _vp]
_lib.mol_profile_step.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int)]
_lib.mol_plan_kernel_configs.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.mol_plan_set_kernel_config.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
_lib.mol_plan_tune_key.argtypes = [_vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_int]



class _SrvInfo(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("finished", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t),
                ("budget", ctypes.c_size_t), ("admit_seconds", ctypes.c_double),
                ("admit_max_seconds", ctypes.c_double), ("round_seconds", ctypes.c_double),
                ("rounds", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("sweeps", ctypes.c_int64)]


SERVER_BATCHED = 1


_lib.mol_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_vp)]
_lib.mol_server_create_ex.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]
_lib.mol_server_destroy.argtypes = [_vp]
_lib.mol_server_submit.argtypes = [_vp, ctypes.POINTER(_Desc), _vp, ctypes.c_int, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64)]
_lib.mol_server_poll.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int)]
_lib.mol_server_result.argtypes = [_vp, ctypes.c_int64, _vp, ctypes.c_int]
_lib.mol_server_stats.argtypes = [_vp, ctypes.POINTER(_SrvInfo)]
_lib.mol_server_last_error.restype = ctypes.c_char_p
for _f in ("mol_plan_kernel_configs", "mol_plan_set_kernel_config", "mol_plan_tune_key",
           "mol_profile_step", "mol_plan_create", "mol_plan_destroy", "mol_plan_get_info", "mol_start", "mol_step",
           "mol_step_source", "mol_solve_source",
           "mol_solve", "mol_solve_prepare", "mol_step_static", "mol_step_bdata", "mol_apply",
           "mol_step_batch",
           "mol_server_create",
           "mol_server_create_ex",
           "mol_server_destroy", "mol_server_submit", "mol_server_poll", "mol_server_result", "mol_server_stats"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTS = ("mol_beta_max", "mol_plan_create", "mol_plan_destroy", "mol_plan_get_info",
           "mol_workspace_bytes", "mol_start", "mol_step", "mol_step_source", "mol_solve",
           "mol_solve_prepare", "mol_step_static", "mol_step_static_max_bytes", "mol_step_bdata",
           "mol_solve_source",
           "mol_step_batch",
           "mol_apply", "mol_profile_step", "mol_plan_kernel_configs",
           "mol_plan_set_kernel_config", "mol_plan_tune_key", "mol_last_error",
           "mol_server_create", "mol_server_create_ex", "mol_server_destroy", "mol_server_submit",
           "mol_server_poll", "mol_server_result", "mol_server_stats", "mol_server_last_error")


def _check(st):
    if st != MOL_OK:
        raise MolError(st, _lib.mol_last_error().decode())


def beta_max(P: int) -> float:
    return float(_lib.mol_beta_max(int(P)))


def last_error() -> str:
    return _lib.mol_last_error().decode()


def make_desc(shape, h, bc=DIRICHLET, P=2, c=1.0, dt=None, cfl=None, beta=0.0, dtype="f64",
              flags=0, mask=None, cross=None):
    """Descriptor for a field of array shape ``shape`` (C order, x last).
    Give either dt or cfl (dt = cfl * h_x / c)."""
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    nx = list(reversed(shape))
    hh = list(h) if np.ndim(h) else [float(h)] * nd
    bb = list(bc) if np.ndim(bc) else [int(bc)] * nd
    if dt is None:
        dt = float(cfl) * hh[0] / c
    d = _Desc()
    d.ndim = nd
    for a in range(3):
        d.n[a] = nx[a] if a < nd else 1
        d.h[a] = float(hh[a]) if a < nd else 1.0
        d.bc[a] = int(bb[a]) if a < nd else 0
    keep = []
    if mask is not None:
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        if nd == 2 and m.shape != shape:
            raise ValueError("mask shape %s does not match the field shape %s" % (m.shape, shape))
        if m.size != int(np.prod(shape)):
            raise ValueError("mask has %d entries for %d nodes" % (m.size, int(np.prod(shape))))
        keep.append(m)
        d.mask = m.ctypes.data
    if cross is not None:
        cr = np.ascontiguousarray(cross, dtype=np.float64)
        if cr.shape != (4,) + shape:
            raise ValueError("cross must have shape (4,) + field shape, got %s" % (cr.shape,))
        keep.append(cr)
        d.cross = cr.ctypes.data
    d.P = int(P)
    d.c = float(c)
    d.dt = float(dt)
    d.beta = float(beta)
    d.dtype = F64 if dtype in ("f64", "float64", F64) else F32
    d.flags = int(flags)
    return d, keep


def workspace_bytes(**kw) -> int:
    d, keep = make_desc(**kw)
    return int(_lib.mol_workspace_bytes(ctypes.byref(d)))


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A solver plan bound to the current device.  Fields are torch tensors of
    the plan's dtype and shape, on that device, contiguous."""

    def __init__(self, shape, h, bc=DIRICHLET, P=2, c=1.0, dt=None, cfl=None, beta=0.0,
                 dtype="f64", flags=0, mask=None, cross=None):
        d, keep = make_desc(shape, h, bc, P, c, dt, cfl, beta, dtype, flags, mask, cross)
        self.shape = tuple(int(s) for s in shape)
        self.fp64 = d.dtype == F64
        self._h = _vp()
        _check(_lib.mol_plan_create(ctypes.byref(d), ctypes.byref(self._h)))
        del keep
        info = _Info()
        _check(_lib.mol_plan_get_info(self._h, ctypes.byref(info)))
        self.info = {
            "beta": info.beta, "beta_max": info.beta_max, "alpha": info.alpha,
            "nu": tuple(info.nu), "points": info.points, "unknowns": info.unknowns,
            "segments": tuple(info.segments), "kernels_per_step": info.kernels_per_step,
            "bytes_per_step": info.bytes_per_step, "workspace_bytes": info.workspace_bytes,
            "kernels_per_source_step": info.kernels_per_source_step,
            "bytes_per_source_step": info.bytes_per_source_step,
        }

    def close(self):
        if self._h:
            _lib.mol_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _t(self, x):
        import torch
        want = torch.float64 if self.fp64 else torch.float32
        if not isinstance(x, torch.Tensor) or x.dtype != want or not x.is_cuda \
                or tuple(x.shape) != self.shape or not x.is_contiguous():
            raise ValueError("expected a contiguous %s CUDA tensor of shape %s" % (want, self.shape))
        return ctypes.c_void_p(x.data_ptr())

    def start(self, u0, u1, stream=None, g=None):
        """u1 = u(dt) from u0 and the initial velocity g (None: zero)."""
        _check(_lib.mol_start(self._h, self._t(u0), None if g is None else self._t(g), self._t(u1),
                              _stream(stream)))

    def step(self, u_prev, u_curr, u_next, stream=None):
        _check(_lib.mol_step(self._h, self._t(u_prev), self._t(u_curr), self._t(u_next),
                             _stream(stream)))

    def step_source(self, u_prev, u_curr, u_next, s_prev, s_curr, s_next, stream=None):
        """One step with the source S at t_{n-1}, t_n, t_{n+1} (s_prev and
        s_next may be None for P = 1)."""
        opt = lambda x: None if x is None else self._t(x)
        _check(_lib.mol_step_source(self._h, self._t(u_prev), self._t(u_curr), self._t(u_next),
                                    opt(s_prev), self._t(s_curr), opt(s_next), _stream(stream)))

    def solve_source(self, u_prev, u_curr, nsteps, G, CG, f, stream=None):
        """nsteps steps in place with the separable source f(t) G(x); f holds
        f(t_{n-1}) .. f(t_{n+nsteps}) (nsteps + 2 values); CG = C[G] (None for
        P = 1)."""
        import numpy as np
        fa = np.ascontiguousarray(f, dtype=np.float64)
        if fa.shape != (int(nsteps) + 2,):
            raise ValueError("f must hold nsteps + 2 values")
        _check(_lib.mol_solve_source(self._h, self._t(u_prev), self._t(u_curr), int(nsteps),
                                     self._t(G), None if CG is None else self._t(CG),
                                     fa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     _stream(stream)))

    def step_bdata(self, u_prev, u_curr, u_next, da, db, next_a=0.0, next_b=0.0, stream=None):
        """One 1D step with boundary data (Dirichlet plans: values; Neumann
        plans: slopes u_x): da, db = even time derivatives d_t^{2j} of the
        data at a and b at t_n, j = 0..P; next_a, next_b = the Dirichlet data
        at t_{n+1} (unused for Neumann)."""
        import numpy as np
        if len(da) != len(db):
            raise ValueError("da and db must hold the same number of derivatives")
        b = np.ascontiguousarray(list(da) + [next_a] + list(db) + [next_b], dtype=np.float64)
        _check(_lib.mol_step_bdata(self._h, self._t(u_prev), self._t(u_curr), self._t(u_next),
                                   b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream)))

    def solve(self, u_prev, u_curr, nsteps, stream=None):
        _check(_lib.mol_solve(self._h, self._t(u_prev), self._t(u_curr), int(nsteps),
                              _stream(stream)))

    def solve_prepare(self, u_prev, u_curr, nsteps, stream=None):
        """Capture the graphs solve(u_prev, u_curr, nsteps) replays, running nothing."""
        _check(_lib.mol_solve_prepare(self._h, self._t(u_prev), self._t(u_curr), int(nsteps),
                                      _stream(stream)))

    def profile_step(self, u_prev, u_curr, u_next, reps=10, stream=None):
        """Per-kernel mean duration (ms) and algorithmic bytes of one step,
        from hipEvents around each launch."""
        mx = 64
        ms = (ctypes.c_double * mx)()
        by = (ctypes.c_double * mx)()
        dr = (ctypes.c_int * mx)()
        ns = (ctypes.c_int * mx)()
        cnt = ctypes.c_int()
        _check(_lib.mol_profile_step(self._h, self._t(u_prev), self._t(u_curr), self._t(u_next),
                                     int(reps), _stream(stream), mx, ms, by, dr, ns,
                                     ctypes.byref(cnt)))
        return [{"ms": ms[i], "bytes": by[i], "dir": "xyz"[dr[i]], "sweeps": ns[i]}
                for i in range(min(cnt.value, mx))]

    def kernel_configs(self, kernel):
        """(valid configuration ids, id in use) of kernel `kernel` of the solve step."""
        ids = (ctypes.c_int * 64)()
        cnt, cur = ctypes.c_int(), ctypes.c_int()
        _check(_lib.mol_plan_kernel_configs(self._h, int(kernel), ids, 64, ctypes.byref(cnt),
                                            ctypes.byref(cur)))
        return [ids[i] for i in range(min(cnt.value, 64))], cur.value

    def set_kernel_config(self, kernel, config):
        _check(_lib.mol_plan_set_kernel_config(self._h, int(kernel), int(config)))

    def tune_key(self, kernel):
        buf = ctypes.create_string_buffer(256)
        _check(_lib.mol_plan_tune_key(self._h, int(kernel), buf, 256))
        return buf.value.decode()

    def apply(self, op, x, out, stream=None):
        code = OPS[op] if isinstance(op, str) else int(op)
        _check(_lib.mol_apply(self._h, code, self._t(x), self._t(out), _stream(stream)))


class Server:
    """Request server (continuous batching of independent solves, admitted by
    device footprint).  batched=True: requests advance in rounds whose sweeps
    of the same kernel run as one batched launch; else every request replays
    its own graph on a stream of the pool.  submit() takes the initial field as
    a host numpy array or a device tensor; the server keeps a reference until
    the result is taken."""

    def __init__(self, budget_bytes, nstreams=4, batched=False):
        h = _vp()
        st = _lib.mol_server_create_ex(int(budget_bytes), int(nstreams),
                                       SERVER_BATCHED if batched else 0, ctypes.byref(h))
        if st != MOL_OK:
            raise MolError(st, _lib.mol_server_last_error().decode())
        self._h = h
        self._keep = {}

    def _chk(self, st):
        if st != MOL_OK:
            raise MolError(st, _lib.mol_server_last_error().decode())

    @staticmethod
    def _field_check(x, shape, want_np, what, need_cuda=None):
        """x must be one contiguous field of the request's shape and dtype."""
        import torch
        want_t = torch.float64 if want_np == np.float64 else torch.float32
        if isinstance(x, np.ndarray):
            if need_cuda:
                raise ValueError("%s must be a CUDA tensor" % what)
            if x.shape != shape:
                raise ValueError("%s has shape %s, expected %s" % (what, x.shape, shape))
            return
        if not isinstance(x, torch.Tensor):
            raise TypeError("%s must be a numpy array or a torch tensor" % what)
        if x.dtype != want_t or tuple(x.shape) != shape or not x.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor of shape %s" % (what, want_t, shape))
        if need_cuda is not None and x.is_cuda != need_cuda:
            raise ValueError("%s must be a %s tensor" % (what, "CUDA" if need_cuda else "host"))
        if x.is_cuda and x.device.index != torch.cuda.current_device():
            raise ValueError("%s is on another device than the server" % what)

    def submit(self, u0, shape, h, nsteps, **kw):
        """Queue a request.  A device u0 is read later on a server stream:
        the producing stream is synchronised here, so the data is complete."""
        shape = tuple(int(x) for x in shape)
        d, keep = make_desc(shape, h, **kw)
        dt = np.float64 if d.dtype == F64 else np.float32
        self._field_check(u0, shape, dt, "u0")
        if isinstance(u0, np.ndarray):
            arr = np.ascontiguousarray(u0, dtype=dt)
            ptr, ondev = arr.ctypes.data, 0
        else:                      # torch tensor: device, or (pinned) host memory
            arr = u0
            ptr, ondev = u0.data_ptr(), 1 if u0.is_cuda else 0
            if u0.is_cuda:
                import torch
                torch.cuda.current_stream().synchronize()
        rid = ctypes.c_int64()
        self._chk(_lib.mol_server_submit(self._h, ctypes.byref(d), ctypes.c_void_p(ptr), ondev,
                                         int(nsteps), ctypes.byref(rid)))
        self._keep[rid.value] = (arr, keep, shape, dt)
        return rid.value

    def poll(self, max_ids=1024):
        ids = (ctypes.c_int64 * max_ids)()
        n = ctypes.c_int()
        self._chk(_lib.mol_server_poll(self._h, ids, max_ids, ctypes.byref(n)))
        return [ids[i] for i in range(n.value)]

    def result(self, rid, out=None):
        """Copies u^nsteps into out (device tensor) or returns a host array."""
        _, _, shape, dt = self._keep[rid]
        if out is None:
            host = np.empty(shape, dtype=dt)
            st = _lib.mol_server_result(self._h, int(rid), ctypes.c_void_p(host.ctypes.data), 0)
            self._keep.pop(rid, None)
            self._chk(st)
            return host
        self._field_check(out, shape, dt, "out", need_cuda=True)
        st = _lib.mol_server_result(self._h, int(rid), ctypes.c_void_p(out.data_ptr()), 1)
        self._keep.pop(rid, None)
        self._chk(st)
        return out

    def stats(self):
        i = _SrvInfo()
        self._chk(_lib.mol_server_stats(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _SrvInfo._fields_}

    def close(self):
        if self._h:
            _lib.mol_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_static(u_prev, u_curr, u_next, shape, h, stream=None, **kw):
    """One step that allocates no device memory (mol_step_static): the plan of
    make_desc(shape, h, **kw), workspace in the library's static array."""
    import torch
    d, keep = make_desc(shape, h, **kw)
    want = torch.float64 if d.dtype == F64 else torch.float32
    for t in (u_prev, u_curr, u_next):
        if not isinstance(t, torch.Tensor) or t.dtype != want or not t.is_cuda \
                or tuple(t.shape) != tuple(int(x) for x in shape) or not t.is_contiguous():
            raise ValueError("expected contiguous %s CUDA tensors of shape %s" % (want, tuple(shape)))
    _check(_lib.mol_step_static(ctypes.byref(d), ctypes.c_void_p(u_prev.data_ptr()),
                                ctypes.c_void_p(u_curr.data_ptr()), ctypes.c_void_p(u_next.data_ptr()),
                                _stream(stream)))


def step_batch(plans, u_prev, u_curr, u_next, stream=None):
    """One step of every plan (mol_step_batch): launches shared across plans
    where they use the same kernel instantiation."""
    n = len(plans)
    if not (len(u_prev) == len(u_curr) == len(u_next) == n):
        raise ValueError("one u_prev, u_curr and u_next per plan")
    arr = lambda xs: (_vp * n)(*xs)  # noqa: E731
    hs = (_vp * n)(*[p.handle for p in plans])
    _check(_lib.mol_step_batch(hs, arr([p._t(t) for p, t in zip(plans, u_prev)]),
                               arr([p._t(t) for p, t in zip(plans, u_curr)]),
                               arr([p._t(t) for p, t in zip(plans, u_next)]), n, _stream(stream)))
