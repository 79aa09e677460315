"""Python binding of libdirprec (directional-preconditioned CFIE solves on MI355X).

Argument marshalling only: every numerical step runs in the HIP library
(`libdirprec.so`, built in-tree by `paper_1408_1578_amd.build`).  The
functions carry the names of the C-ABI in include/dirprec.h.  Device arrays
are torch complex128 CUDA tensors laid out as (nrhs, n) (i.e. column-major
n x nrhs); torch is used for device memory and the stream only.

Importing this package does not need a GPU; loading the library does not
either, but every compute call does.  If the library is missing the calls
raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdirprec.so")

DP_OK, DP_ENOCONV = 0, 1
DP_EINVAL, DP_ENOMEM, DP_EDEVICE, DP_ESINGULAR, DP_ESTATE = -1, -2, -3, -4, -5
DP_SOFT, DP_HARD = 0, 1
DP_OP_S, DP_OP_D, DP_OP_DP, DP_OP_DS = 2, 3, 4, 5

# every symbol declared in include/dirprec.h
EXPORTED = [
    "dp_ctx_create", "dp_ctx_destroy", "dp_last_error", "dp_problem_create",
    "dp_problem_destroy", "dp_problem_kappa", "dp_rhs_plane_wave", "dp_matvec", "dp_matvec_mixed", "dp_layer_apply",
    "dp_precond_build", "dp_precond_apply", "dp_precond_apply_mixed", "dp_precond_apply_noalloc",
    "dp_precond_get_info", "dp_precond_export",
    "dp_solve", "dp_hankel_dev", "dp_hankel_host", "dp_dense_lu_test",
    "dp_autotune", "dp_server_create", "dp_server_submit", "dp_server_wait", "dp_server_get_stats", "dp_server_destroy",
]


class DpError(RuntimeError):
    def __init__(self, func, code, msg):
        super().__init__(f"{func} failed with code {code}: {msg}")
        self.code = code


class PrecondOpts(ctypes.Structure):
    _fields_ = [("m_ell", ctypes.c_double), ("min_pts", ctypes.c_int),
                ("m_c", ctypes.c_int), ("t_keep", ctypes.c_double), ("w_solver", ctypes.c_int),
                ("graphs", ctypes.c_int), ("gj_steps", ctypes.c_int)]


class PrecondInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n_classes", ctypes.c_int64), ("NW", ctypes.c_int64),
                ("nnzE", ctypes.c_int64), ("nnzW", ctypes.c_int64), ("nnzLU", ctypes.c_int64),
                ("levels", ctypes.c_int64), ("t_setup", ctypes.c_double), ("dense_w", ctypes.c_int64)]


DP_PREC_FP64, DP_PREC_MIXED = 0, 1


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int),
                ("max_iters", ctypes.c_int), ("use_precond", ctypes.c_int),
                ("precision", ctypes.c_int), ("inner_tol", ctypes.c_double), ("eager", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters_max", ctypes.c_int64), ("matvecs", ctypes.c_int64),
                ("applies", ctypes.c_int64), ("relres_max", ctypes.c_double),
                ("t_total", ctypes.c_double), ("t_matvec", ctypes.c_double),
                ("t_apply", ctypes.c_double), ("t_krylov", ctypes.c_double),
                ("sweep_launches", ctypes.c_int64), ("t_sweep", ctypes.c_double),
                ("refinements", ctypes.c_int64), ("matvecs_fp32", ctypes.c_int64),
                ("sweep_launches_fp32", ctypes.c_int64), ("t_sweep_fp32", ctypes.c_double)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("t_default_ms", ctypes.c_double), ("t_best_ms", ctypes.c_double),
                ("target_blocks", ctypes.c_int64), ("matrix_cores", ctypes.c_int64), ("candidates", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("mem_budget", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("xy", ctypes.c_void_p), ("nrm", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("kappa", ctypes.c_void_p), ("omega", ctypes.c_double),
                ("eta", ctypes.c_double), ("kind", ctypes.c_int), ("nrhs", ctypes.c_int64),
                ("angles", ctypes.c_void_p), ("f", ctypes.c_void_p), ("solve", SolveOpts)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("mem_estimate", ctypes.c_int64), ("slot", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "failed", "running", "queued",
                                              "mem_in_use", "mem_budget", "mem_peak")]


_lib = None


def lib():
    """Load libdirprec.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    # torch ships its own HIP runtime under the same soname; initialise it first
    # so that the library binds to that one copy (one runtime per process).
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "dp_ctx_create": (ci, [ci, vp, pp]),
        "dp_ctx_destroy": (None, [vp]),
        "dp_last_error": (ctypes.c_char_p, []),
        "dp_problem_create": (ci, [vp, i64, vp, vp, vp, vp, dbl, dbl, ci, pp]),
        "dp_problem_destroy": (None, [vp]),
        "dp_problem_kappa": (ci, [vp, vp]),
        "dp_rhs_plane_wave": (ci, [vp, i64, vp, vp]),
        "dp_matvec": (ci, [vp, i64, vp, vp]),
        "dp_matvec_mixed": (ci, [vp, i64, vp, vp]),
        "dp_layer_apply": (ci, [vp, ci, i64, vp, vp]),
        "dp_precond_build": (ci, [vp, ctypes.POINTER(PrecondOpts)]),
        "dp_precond_apply": (ci, [vp, i64, vp, vp]),
        "dp_precond_apply_mixed": (ci, [vp, i64, vp, vp]),
        "dp_precond_apply_noalloc": (ci, [vp, i64, vp, vp]),
        "dp_precond_get_info": (ci, [vp, ctypes.POINTER(PrecondInfo)]),
        "dp_precond_export": (ci, [vp, vp, vp, vp, vp]),
        "dp_solve": (ci, [vp, i64, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp, vp]),
        "dp_hankel_dev": (ci, [vp, i64, vp, vp]),
        "dp_hankel_host": (ci, [i64, vp, vp]),
        "dp_dense_lu_test": (ci, [vp, i64, vp, vp, vp]),
        "dp_autotune": (ci, [vp, i64, ci, ctypes.POINTER(TuneInfo)]),
        "dp_server_create": (ci, [ci, ctypes.POINTER(ServerOpts), pp]),
        "dp_server_submit": (ci, [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_int64)]),
        "dp_server_wait": (ci, [vp, i64, vp, ctypes.POINTER(SolveInfo), ctypes.POINTER(RequestTimes)]),
        "dp_server_get_stats": (ci, [vp, ctypes.POINTER(ServerStats)]),
        "dp_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(name, rc, allow=()):
    if rc < 0 and rc not in allow:
        raise DpError(name, rc, lib().dp_last_error().decode())
    return rc


def _ptr(t, ctx):
    """Device pointer of a contiguous torch tensor on the context's GPU."""
    if not getattr(t, "is_cuda", False):
        raise ValueError("expected a torch tensor in device memory")
    if t.device.index != ctx.device:
        raise ValueError(f"tensor is on device {t.device.index}, the context on device {ctx.device}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _cols(t, n):
    if t.dtype.__str__() != "torch.complex128":
        raise TypeError("expected a complex128 tensor")
    if t.dim() == 1:
        if t.shape[0] != n:
            raise ValueError("length mismatch")
        return 1
    if t.dim() != 2 or t.shape[1] != n:
        raise ValueError("expected shape (nrhs, n)")
    return t.shape[0]


def _host(a, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- context
class Context:
    def __init__(self, device: int = 0, stream=None):
        h = ctypes.c_void_p()
        s = None if stream is None else ctypes.c_void_p(stream)
        _check("dp_ctx_create", lib().dp_ctx_create(device, s, ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().dp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dp_ctx_create(device=0, stream=None):
    return Context(device, stream)


def dp_ctx_destroy(ctx):
    ctx.close()


# ---------------------------------------------------------------- problem
class Problem:
    def __init__(self, ctx, x, nu, w, kappa, omega, eta, kind):
        n = int(np.asarray(w).size)
        xa, xp = _host(np.asarray(x).reshape(n, 2))
        na, np_ = _host(np.asarray(nu).reshape(n, 2))
        wa, wp = _host(w)
        ka, kp = (None, None) if kappa is None else _host(kappa)  # None: computed by the library
        h = ctypes.c_void_p()
        _check("dp_problem_create", lib().dp_problem_create(ctx.h, n, xp, np_, wp, kp, float(omega),
                                                            float(eta), int(kind), ctypes.byref(h)))
        self.h, self.n, self.kind, self.ctx = h, n, kind, ctx
        self.omega, self.eta = float(omega), float(eta)

    @classmethod
    def from_boundary(cls, ctx, b, omega, eta, kind):
        return cls(ctx, b.x, b.nu, b.w, b.kappa, omega, eta, kind)

    def close(self):
        if self.h:
            lib().dp_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dp_problem_create(ctx, x, nu, w, kappa, omega, eta, kind):
    return Problem(ctx, x, nu, w, kappa, omega, eta, kind)


def dp_problem_destroy(p):
    p.close()


def dp_problem_kappa(p):
    """The curvatures the problem uses, (n,) float64."""
    k = np.empty(p.n, np.float64)
    _check("dp_problem_kappa", lib().dp_problem_kappa(p.h, k.ctypes.data_as(ctypes.c_void_p)))
    return k


def dp_rhs_plane_wave(p, angles, f):
    a, ap = _host(np.atleast_1d(angles))
    nr = _cols(f, p.n)
    if nr != a.size:
        raise ValueError("angles / columns mismatch")
    _check("dp_rhs_plane_wave", lib().dp_rhs_plane_wave(p.h, nr, ap, _ptr(f, p.ctx)))


def dp_matvec(p, q, y):
    nr = _cols(q, p.n)
    if _cols(y, p.n) != nr:
        raise ValueError("shape mismatch")
    _check("dp_matvec", lib().dp_matvec(p.h, nr, _ptr(q, p.ctx), _ptr(y, p.ctx)))


def dp_matvec_mixed(p, q, y):
    nr = _cols(q, p.n)
    if _cols(y, p.n) != nr:
        raise ValueError("shape mismatch")
    _check("dp_matvec_mixed", lib().dp_matvec_mixed(p.h, nr, _ptr(q, p.ctx), _ptr(y, p.ctx)))


def dp_layer_apply(p, op, q, y):
    nr = _cols(q, p.n)
    if _cols(y, p.n) != nr:
        raise ValueError("shape mismatch")
    _check("dp_layer_apply", lib().dp_layer_apply(p.h, int(op), nr, _ptr(q, p.ctx), _ptr(y, p.ctx)))


W_AUTO, W_SPARSE, W_DENSE = 0, 1, 2


def dp_precond_build(p, m_ell=4.0, min_pts=8, m_c=10, t_keep=3.0, w_solver=W_AUTO, graphs=True, gj_steps=0):
    o = PrecondOpts(m_ell, min_pts, m_c, t_keep, int(w_solver), 1 if graphs else 0, int(gj_steps))
    _check("dp_precond_build", lib().dp_precond_build(p.h, ctypes.byref(o)))


def dp_precond_apply(p, v, z):
    nr = _cols(v, p.n)
    if _cols(z, p.n) != nr:
        raise ValueError("shape mismatch")
    _check("dp_precond_apply", lib().dp_precond_apply(p.h, nr, _ptr(v, p.ctx), _ptr(z, p.ctx)))


def dp_precond_apply_mixed(p, v, z):
    nr = _cols(v, p.n)
    if _cols(z, p.n) != nr:
        raise ValueError("shape mismatch")
    _check("dp_precond_apply_mixed", lib().dp_precond_apply_mixed(p.h, nr, _ptr(v, p.ctx), _ptr(z, p.ctx)))


def dp_precond_apply_noalloc(p, v, z):
    nr = _cols(v, p.n)
    if _cols(z, p.n) != nr:
        raise ValueError("shape mismatch")
    _check("dp_precond_apply_noalloc", lib().dp_precond_apply_noalloc(p.h, nr, _ptr(v, p.ctx), _ptr(z, p.ctx)))


def dp_precond_get_info(p):
    info = PrecondInfo()
    _check("dp_precond_get_info", lib().dp_precond_get_info(p.h, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in PrecondInfo._fields_}


def dp_precond_export(p):
    info = dp_precond_get_info(p)
    m = info["m"]
    off = np.zeros(m, np.int64)
    ln = np.zeros(m, np.int64)
    ei = np.zeros(4 * m * (m - 1), np.int64)
    ev = np.zeros(2 * m * (m - 1), np.float64)
    _check("dp_precond_export", lib().dp_precond_export(
        p.h, off.ctypes.data_as(ctypes.c_void_p), ln.ctypes.data_as(ctypes.c_void_p),
        ei.ctypes.data_as(ctypes.c_void_p), ev.ctypes.data_as(ctypes.c_void_p)))
    return off, ln, ei.reshape(-1, 4), ev.view(np.complex128)


def dp_solve(p, f, q, tol=1e-8, restart=80, max_iters=2000, use_precond=False, precision=DP_PREC_FP64,
             inner_tol=0.0, eager=False):
    nr = _cols(f, p.n)
    if _cols(q, p.n) != nr:
        raise ValueError("shape mismatch")
    o = SolveOpts(tol, restart, max_iters, 1 if use_precond else 0, int(precision), inner_tol, 1 if eager else 0)
    info = SolveInfo()
    its = np.zeros(nr, np.int64)
    rel = np.zeros(nr, np.float64)
    rc = _check("dp_solve", lib().dp_solve(p.h, nr, _ptr(f, p.ctx), _ptr(q, p.ctx), ctypes.byref(o), ctypes.byref(info),
                                           its.ctypes.data_as(ctypes.c_void_p),
                                           rel.ctypes.data_as(ctypes.c_void_p)))
    out = {f_: getattr(info, f_) for f_, _ in SolveInfo._fields_}
    out["converged"] = rc == DP_OK
    out["iters"] = its
    out["relres"] = rel
    return out


def dp_autotune(p, nrhs, precision=DP_PREC_FP64):
    info = TuneInfo()
    _check("dp_autotune", lib().dp_autotune(p.h, int(nrhs), int(precision), ctypes.byref(info)))
    return {f_: getattr(info, f_) for f_, _ in TuneInfo._fields_}


def dp_hankel_dev(ctx, z, out):
    _check("dp_hankel_dev", lib().dp_hankel_dev(ctx.h, z.numel(), _ptr(z, ctx), _ptr(out, ctx)))


def dp_hankel_host(z):
    za, zp = _host(np.atleast_1d(z))
    out = np.zeros(4 * za.size)
    _check("dp_hankel_host", lib().dp_hankel_host(za.size, zp, out.ctypes.data_as(ctypes.c_void_p)))
    out = out.reshape(-1, 4)
    return out[:, 0] + 1j * out[:, 1], out[:, 2] + 1j * out[:, 3]


def dp_dense_lu_test(ctx, a):
    """Dense device LU of the (n, n) complex matrix a: (rc, lu, perm) with
    lu = L below the diagonal (unit) and U on and above, a[perm] = L U;
    rc is DP_OK or DP_ESINGULAR (other errors raise)."""
    a = np.asfortranarray(np.asarray(a, np.complex128))
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("square matrix expected")
    lu = np.zeros((n, n), np.complex128, order="F")
    perm = np.zeros(n, np.int64)
    rc = lib().dp_dense_lu_test(ctx.h, n, a.ctypes.data_as(ctypes.c_void_p), lu.ctypes.data_as(ctypes.c_void_p),
                                perm.ctypes.data_as(ctypes.c_void_p))
    _check("dp_dense_lu_test", rc, allow=(DP_ESINGULAR,))
    return rc, lu, perm


class Server:
    """Request server (dp_server_*): independent solves admitted onto the GPU
    as worker slots and device memory free up; submit() returns at once,
    wait() blocks (the GIL is released while it waits)."""

    def __init__(self, device=0, slots=4, mem_budget=0):
        self.h = ctypes.c_void_p()
        o = ServerOpts(int(slots), int(mem_budget))
        _check("dp_server_create", lib().dp_server_create(int(device), ctypes.byref(o), ctypes.byref(self.h)))
        self._n = {}

    def submit(self, b, omega, eta, kind, angles=None, f=None, tol=1e-8, restart=80, max_iters=2000,
               use_precond=True, precision=DP_PREC_FP64, inner_tol=0.0):
        """b: boundary with x (n, 2), nu (n, 2), w (n,), kappa (n,) or None.  angles: plane-wave angles, or
        f: (n, nrhs) complex data.  Returns the request id."""
        xy, xyp = _host(b.x)
        nu, nup = _host(b.nu)
        w, wp = _host(b.w)
        ka, kap = (None, None) if b.kappa is None else _host(b.kappa)
        n = w.size
        if angles is not None:
            an, anp = _host(np.atleast_1d(angles))
            nrhs, fp = an.size, None
        else:
            fa = np.asarray(f, np.complex128)
            fa = fa[:, None] if fa.ndim == 1 else fa
            nrhs = fa.shape[1]
            fc, fp = _host(np.asfortranarray(fa).ravel(order="F").view(np.float64))
            anp = None
        r = Request(n, xyp, nup, wp, kap, float(omega), float(eta), int(kind), nrhs, anp, fp,
                    SolveOpts(tol, restart, max_iters, 1 if use_precond else 0, int(precision), inner_tol, 0))
        rid = ctypes.c_int64()
        _check("dp_server_submit", lib().dp_server_submit(self.h, ctypes.byref(r), ctypes.byref(rid)))
        self._n[rid.value] = (n, nrhs)
        return rid.value

    def wait(self, rid):
        """(q (n, nrhs) complex, solve info dict, times dict, status)."""
        n, nrhs = self._n.pop(rid, (0, 0))  # unknown ids: the library reports them
        q = np.zeros(max(1, 2 * n * nrhs))
        info, t = SolveInfo(), RequestTimes()
        rc = _check("dp_server_wait", lib().dp_server_wait(self.h, int(rid), q.ctypes.data_as(ctypes.c_void_p)
                                                           if n else None, ctypes.byref(info), ctypes.byref(t)))
        out = {f_: getattr(info, f_) for f_, _ in SolveInfo._fields_}
        out["converged"] = rc == DP_OK
        times = {f_: getattr(t, f_) for f_, _ in RequestTimes._fields_}
        return q.view(np.complex128).reshape(nrhs, n).T, out, times, rc

    def stats(self):
        st = ServerStats()
        _check("dp_server_get_stats", lib().dp_server_get_stats(self.h, ctypes.byref(st)))
        return {f_: getattr(st, f_) for f_, _ in ServerStats._fields_}

    def close(self):
        if self.h:
            lib().dp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
