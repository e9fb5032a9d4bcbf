"""Thin ctypes binding of ``libnlth.so`` (the C-ABI declared in include/nlth.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  The module-level ``nlth_*`` functions mirror the C entry points
one to one; :class:`Context` and :class:`Ensemble` are conveniences built on
them.  PyTorch, when present, only supplies the compute stream (the current
``torch.cuda`` stream) so the library's work orders with torch's.

Loading fails loudly if the library has not been built
(``python -m paper_2604_02755_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlth.so")

NLTH_OK = 0
NLTH_EINVAL = -1
NLTH_EDEVICE = -2
NLTH_ENOMEM_DEVICE = -3
NLTH_ENOMEM_HOST = -4
NLTH_ENOCONV = -5
NLTH_EBUSY = -6
NLTH_ECANCELED = -7
NLTH_ETIMEDOUT = -8
NLTH_ENOTFOUND = -9
NLTH_FP64, NLTH_MIXED = 0, 1
NLTH_INNER_BF16, NLTH_INNER_FP32, NLTH_INNER_BF16_MEAN = 0, 1, 2
INNER_CG, INNER_CHEBYSHEV = 0, 1  # nlth_tuning.inner_method
NLTH_SPEC_VELOCITY, NLTH_SPEC_PSEUDO_VELOCITY = 0, 1
NLTH_OP_A, NLTH_OP_K, NLTH_OP_M, NLTH_OP_DIAG = 0, 1, 2, 3
NLTH_DEVICE_NONE = -1

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class nlth_ctx_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("host_budget", C.c_int64), ("stream", C.c_void_p),
                ("log_level", C.c_int32), ("max_batch", C.c_int32), ("paging_sets", C.c_int32)]


class nlth_mesh_desc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("xyz", _dp), ("n_tets", C.c_int32), ("tet10", _ip),
                ("layer", _ip), ("n_bfaces", C.c_int32), ("bface6", _ip),
                ("bface_kind", C.POINTER(C.c_uint8)), ("n_recv", C.c_int32), ("recv", _ip)]


class nlth_mesh_info(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_tets", C.c_int32), ("n_colors", C.c_int32),
                ("n_bnodes", C.c_int32), ("volume", C.c_double), ("n_clusters", C.c_int32),
                ("cluster_rows", C.c_int64)]


class nlth_problem(C.Structure):
    _fields_ = [("n_members", C.c_int32), ("n_layers", C.c_int32), ("rho", _dp), ("vs", _dp),
                ("nu", _dp), ("gamma_ref", _dp), ("h_max", _dp), ("nonlinear", _ip),
                ("n_springs", C.c_int32), ("dirs", _dp), ("weights", _dp),
                ("damping_mode", C.c_int32), ("h0", C.c_double), ("f_lo", C.c_double),
                ("f_hi", C.c_double), ("dt", C.c_double), ("n_steps", C.c_int32),
                ("input_acc", _dp), ("cg_tol", C.c_double), ("cg_maxit", C.c_int32),
                ("precision", C.c_int32), ("inner_tol", C.c_double), ("inner_maxit", C.c_int32),
                ("inner_dtype", C.c_int32), ("masing_depth", C.c_int32)]


class nlth_tuning(C.Structure):
    _fields_ = [("ebe_block", C.c_int32), ("check_every", C.c_int32), ("use_graph", C.c_int32),
                ("inner_maxit", C.c_int32), ("inner_tol", C.c_double), ("scatter", C.c_int32),
                ("cluster_blocks", C.c_int32), ("inner_method", C.c_int32), ("zero_copy", C.c_int32),
                ("tail_members", C.c_int32), ("predictor", C.c_int32)]


class nlth_result(C.Structure):
    _fields_ = [("vel", _dp), ("iters", _ip), ("member_status", _ip), ("vmax", _dp)]


class nlth_stats(C.Structure):
    _fields_ = [("steps_done", C.c_int32), ("paged", C.c_int32), ("outer_iters", C.c_int64),
                ("inner_iters", C.c_int64), ("ms_total", C.c_double), ("ms_ebe64", C.c_double),
                ("ms_ebe32", C.c_double), ("ms_vec", C.c_double), ("ms_law", C.c_double),
                ("ms_other", C.c_double), ("n_ebe64", C.c_int64), ("n_ebe32", C.c_int64),
                ("n_law", C.c_int64), ("elems_ebe64", C.c_int64), ("elems_ebe32", C.c_int64),
                ("h2d_bytes", C.c_int64), ("d2h_bytes", C.c_int64), ("ms_copy", C.c_double),
                ("n_members", C.c_int32), ("members_padded", C.c_int32), ("n_colors", C.c_int32),
                ("device_bytes", C.c_int64), ("host_bytes", C.c_int64), ("ms_gather32", C.c_double),
                ("n_gather32", C.c_int64), ("cheb_lo_min", C.c_double), ("cheb_hi_max", C.c_double),
                ("ms_tail32", C.c_double), ("n_tail32", C.c_int64), ("elems_tail32", C.c_int64),
                ("member_sets", C.c_int32)]


EXPORTS = {
    "nlth_version": (C.c_int, []),
    "nlth_last_error": (C.c_char_p, [C.c_void_p]),
    "nlth_ctx_create": (C.c_int, [C.c_int, C.POINTER(nlth_ctx_opts), C.POINTER(C.c_void_p)]),
    "nlth_ctx_destroy": (C.c_int, [C.c_void_p]),
    "nlth_mesh_create": (C.c_int, [C.c_void_p, C.POINTER(nlth_mesh_desc), C.POINTER(C.c_void_p)]),
    "nlth_mesh_destroy": (C.c_int, [C.c_void_p]),
    "nlth_mesh_query": (C.c_int, [C.c_void_p, C.POINTER(nlth_mesh_info), _ip, _ip]),
    "nlth_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(nlth_problem), C.POINTER(nlth_result)]),
    "nlth_ens_create": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(nlth_problem), C.POINTER(C.c_void_p)]),
    "nlth_ens_step": (C.c_int, [C.c_void_p, C.c_int32]),
    "nlth_ens_read": (C.c_int, [C.c_void_p, C.POINTER(nlth_result)]),
    "nlth_ens_destroy": (C.c_int, [C.c_void_p]),
    "nlth_ens_stats": (C.c_int, [C.c_void_p, C.POINTER(nlth_stats)]),
    "nlth_ens_set_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "nlth_ens_reset_stats": (C.c_int, [C.c_void_p]),
    "nlth_ens_set_tuning": (C.c_int, [C.c_void_p, C.c_void_p]),
    "nlth_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(nlth_problem), C.POINTER(nlth_result),
                              C.POINTER(C.c_uint64)]),
    "nlth_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)]),
    "nlth_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_double]),
    "nlth_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "nlth_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "nlth_apply_operator": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(nlth_problem), C.c_int32,
                                      C.c_int32, _dp, _dp, _dp, _dp]),
    "nlth_response_spectra": (C.c_int, [C.c_void_p, _dp, C.c_int32, C.c_int32, C.c_double, _dp, C.c_int32,
                                        C.c_double, C.c_int32, _dp]),
    "nlth_apply_operator_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(nlth_problem), C.c_int32,
                                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None


def lib():
    """Load libnlth.so (raises if it is missing: no CPU fallback exists).

    PyTorch, when installed, is imported first: its wheel carries its own HIP
    runtime, and a process must hold only one.  Loaded after torch, the
    library binds to torch's runtime (same soname); loaded before it, torch
    would bring a second HIP/HSA runtime that cannot open the device again."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2604_02755_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class NlthError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nlth error {code}: {msg}")
        self.code = code


def _check(rc, ctx=None):
    if rc != NLTH_OK:
        msg = lib().nlth_last_error(ctx)
        raise NlthError(rc, msg.decode() if msg else "")
    return rc


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


# ---------------------------------------------------------------------------
# same-name wrappers
# ---------------------------------------------------------------------------

def nlth_version() -> int:
    return lib().nlth_version()


def nlth_ctx_create(device: int = 0, hbm_budget: int = 0, host_budget: int = 0, stream=None,
                    log_level: int = 0, max_batch: int = 0, paging_sets: int = 0):
    opts = nlth_ctx_opts(int(hbm_budget), int(host_budget), stream, int(log_level), int(max_batch),
                         int(paging_sets))
    h = C.c_void_p()
    _check(lib().nlth_ctx_create(int(device), C.byref(opts), C.byref(h)))
    return h


def nlth_ctx_destroy(ctx):
    return _check(lib().nlth_ctx_destroy(ctx))


def _mesh_desc(mesh, keep):
    xyz = _f64(mesh.xyz)
    tet = _i32(mesh.tet10)
    lay = _i32(mesh.layer)
    bf = _i32(mesh.bface6)
    bk = np.ascontiguousarray(mesh.bface_kind, dtype=np.uint8)
    rc = _i32(mesh.recv)
    keep += [xyz, tet, lay, bf, bk, rc]
    return nlth_mesh_desc(int(xyz.shape[0]), _ptr(xyz), int(tet.shape[0]), _ptr(tet, _ip), _ptr(lay, _ip),
                          int(bf.shape[0]), _ptr(bf, _ip), bk.ctypes.data_as(C.POINTER(C.c_uint8)),
                          int(rc.size), _ptr(rc, _ip))


def nlth_mesh_create(ctx, mesh):
    keep = []
    d = _mesh_desc(mesh, keep)
    h = C.c_void_p()
    _check(lib().nlth_mesh_create(ctx, C.byref(d), C.byref(h)), ctx)
    return h


def nlth_mesh_destroy(mesh_h):
    return lib().nlth_mesh_destroy(mesh_h)


def nlth_mesh_query(ctx, mesh_h, n_tets: int, n_colors_max: int = 256):
    info = nlth_mesh_info()
    order = np.zeros(n_tets, np.int32)
    off = np.zeros(n_colors_max + 1, np.int32)
    _check(lib().nlth_mesh_query(mesh_h, C.byref(info), _ptr(order, _ip), _ptr(off, _ip)), ctx)
    return info, order, off[: info.n_colors + 1]


def _problem_struct(prob, keep, members=None, n_steps=None):
    """nlth_problem from the problem's arrays; the shapes the library reads
    are checked here (a short array would otherwise be read past its end)."""
    sel = slice(None) if members is None else members
    rho = _f64(np.asarray(prob.rho)[sel])
    vs = _f64(np.asarray(prob.vs)[sel])
    nu = _f64(np.asarray(prob.nu)[sel])
    gr = _f64(np.asarray(prob.gamma_ref)[sel])
    hm = _f64(prob.h_max)
    nl = _i32(prob.nonlinear)
    dirs = _f64(prob.dirs)
    w = _f64(prob.weights)
    ns = int(prob.n_steps if n_steps is None else n_steps)
    acc_all = np.asarray(prob.input_acc)[sel]
    if rho.ndim != 2:
        raise ValueError(f"rho must be [n_members, n_layers], got shape {rho.shape}")
    nm, nly = rho.shape
    for name, a in (("vs", vs), ("nu", nu), ("gamma_ref", gr)):
        if a.shape != (nm, nly):
            raise ValueError(f"{name} must have shape {(nm, nly)} like rho, got {a.shape}")
    if hm.shape != (nly,) or nl.shape != (nly,):
        raise ValueError(f"h_max and nonlinear must have {nly} entries (one per layer), got {hm.shape}, {nl.shape}")
    if dirs.ndim != 2 or dirs.shape[1] != 6 or w.shape != (dirs.shape[0],):
        raise ValueError(f"dirs must be [n_springs, 6] and weights [n_springs], got {dirs.shape}, {w.shape}")
    if ns < 0 or acc_all.ndim != 3 or acc_all.shape[0] != nm or acc_all.shape[1] < ns or acc_all.shape[2] != 3:
        raise ValueError(f"input_acc must be [n_members={nm}, >= n_steps={ns}, 3], got {acc_all.shape}")
    acc = _f64(acc_all[:, :ns])
    keep += [rho, vs, nu, gr, hm, nl, dirs, w, acc]
    return nlth_problem(int(rho.shape[0]), int(rho.shape[1]), _ptr(rho), _ptr(vs), _ptr(nu), _ptr(gr),
                        _ptr(hm), _ptr(nl, _ip), int(dirs.shape[0]), _ptr(dirs), _ptr(w),
                        int(prob.damping_mode), float(prob.h0), float(prob.f_lo), float(prob.f_hi),
                        float(prob.dt), ns, _ptr(acc), float(prob.cg_tol), int(prob.cg_maxit),
                        int(prob.precision), float(prob.inner_tol), int(prob.inner_maxit),
                        int(getattr(prob, "inner_dtype", 0)), int(getattr(prob, "masing_depth", 1)))


def _result_buffers(nm, ns, nrecv):
    out = dict(vel=np.zeros((nm, ns, nrecv, 3)), iters=np.zeros((nm, ns, 2), np.int32),
               status=np.zeros(nm, np.int32), vmax=np.zeros((nm, nrecv)))
    res = nlth_result(_ptr(out["vel"]), _ptr(out["iters"], _ip), _ptr(out["status"], _ip), _ptr(out["vmax"]))
    return out, res


def nlth_solve(ctx, mesh_h, mesh, prob, n_steps=None, members=None):
    """Whole-run solve; returns dict(vel [nm, ns, nrecv, 3], iters, status, vmax, rc)."""
    keep = []
    p = _problem_struct(prob, keep, members, n_steps)
    out, res = _result_buffers(p.n_members, p.n_steps, int(np.asarray(mesh.recv).size))
    rc = lib().nlth_solve(ctx, mesh_h, C.byref(p), C.byref(res))
    out["rc"] = rc
    if rc not in (NLTH_OK, NLTH_ENOCONV):
        _check(rc, ctx)
    return out


def nlth_response_spectra(ctx, vel, dt, periods, h=0.05, kind=0):
    """Velocity response spectra of records vel [n_series, n_steps] (or one
    record); returns [n_series, n_periods]."""
    v = _f64(vel)
    v = v.reshape(1, -1) if v.ndim == 1 else v
    T = _f64(periods).reshape(-1)
    out = np.zeros((v.shape[0], T.size))
    _check(lib().nlth_response_spectra(ctx, _ptr(v), int(v.shape[0]), int(v.shape[1]), float(dt), _ptr(T),
                                       int(T.size), float(h), int(kind), _ptr(out)), ctx)
    return out


def nlth_apply_operator(ctx, mesh_h, prob, which, precision, D_ip, h, x):
    keep = []
    p = _problem_struct(prob, keep, [0], 0)
    D = _f64(D_ip)
    hh = _f64(h) if h is not None else None
    xx = _f64(x)
    y = np.zeros_like(xx)
    _check(lib().nlth_apply_operator(ctx, mesh_h, C.byref(p), int(which), int(precision), _ptr(D),
                                     _ptr(hh), _ptr(xx), _ptr(y)), ctx)
    return y


def nlth_apply_operator_noalloc(ctx, mesh_h, prob, which, D_ptr, h_ptr, x_ptr, y_ptr):
    """FP64 y = Op x on device buffers (addresses as integers; h_ptr may be 0),
    queued on the context's stream with no allocation; returns once queued."""
    keep = []
    p = _problem_struct(prob, keep, [0], 0)
    _check(lib().nlth_apply_operator_noalloc(ctx, mesh_h, C.byref(p), int(which), C.c_void_p(int(D_ptr)),
                                             C.c_void_p(int(h_ptr)) if h_ptr else None, C.c_void_p(int(x_ptr)),
                                             C.c_void_p(int(y_ptr))), ctx)


# ---------------------------------------------------------------------------
# conveniences
# ---------------------------------------------------------------------------

def torch_stream():
    """The current torch.cuda stream handle, or None when torch/ROCm is absent."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class Ensemble:
    """Staged solve: create (uploads everything), step, read, stats."""

    def __init__(self, ctx, mesh_h, mesh, prob, members=None, n_steps=None):
        self.ctx = ctx
        self._keep = []
        self.p = _problem_struct(prob, self._keep, members, n_steps)
        self.nrecv = int(np.asarray(mesh.recv).size)
        self.h = C.c_void_p()
        _check(lib().nlth_ens_create(ctx, mesh_h, C.byref(self.p), C.byref(self.h)), ctx)

    def step(self, n):
        return _check(lib().nlth_ens_step(self.h, int(n)), self.ctx)

    def read(self):
        out, res = _result_buffers(self.p.n_members, self.p.n_steps, self.nrecv)
        _check(lib().nlth_ens_read(self.h, C.byref(res)), self.ctx)
        return out

    def stats(self):
        st = nlth_stats()
        _check(lib().nlth_ens_stats(self.h, C.byref(st)), self.ctx)
        return {k: getattr(st, k) for k, _ in nlth_stats._fields_}

    def set_profile(self, on=True):
        lib().nlth_ens_set_profile(self.h, int(bool(on)))

    def reset_stats(self):
        lib().nlth_ens_reset_stats(self.h)

    def set_tuning(self, ebe_block=0, check_every=0, use_graph=-1, inner_maxit=0, inner_tol=0.0, scatter=-1,
                   cluster_blocks=0, inner_method=-1, zero_copy=-1, tail_members=-1, predictor=-1):
        """nlth_ens_set_tuning: the defaults (0, or -1 where 0 is a setting) keep
        the current value; include/nlth.h documents each field."""
        t = nlth_tuning(int(ebe_block), int(check_every), int(use_graph), int(inner_maxit), float(inner_tol),
                        int(scatter), int(cluster_blocks), int(inner_method), int(zero_copy), int(tail_members),
                        int(predictor))
        return _check(lib().nlth_ens_set_tuning(self.h, C.byref(t)), self.ctx)

    def close(self):
        if self.h:
            lib().nlth_ens_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    def __init__(self, device=0, hbm_budget=0, host_budget=0, use_torch_stream=True, max_batch=0, paging_sets=0):
        stream = torch_stream() if (use_torch_stream and device != NLTH_DEVICE_NONE) else None
        self._stream = stream
        self.h = nlth_ctx_create(device, hbm_budget, host_budget, stream, 0, max_batch, paging_sets)
        self._meshes = []

    def mesh(self, mesh):
        mh = nlth_mesh_create(self.h, mesh)
        self._meshes.append(mh)
        return mh

    def solve(self, mesh_h, mesh, prob, **kw):
        return nlth_solve(self.h, mesh_h, mesh, prob, **kw)

    def solve_as_served(self, mesh_h, mesh, prob):
        """The problem solved alone with the policy of the serving batches (the
        quadratic-extrapolation initial guess): a served request's results
        equal these up to the order of reductions."""
        ens = self.ensemble(mesh_h, mesh, prob)
        try:
            ens.set_tuning(predictor=2)
            ens.step(prob.n_steps)
            return ens.read()
        finally:
            ens.close()

    def ensemble(self, mesh_h, mesh, prob, **kw):
        return Ensemble(self.h, mesh_h, mesh, prob, **kw)

    def apply_operator(self, mesh_h, prob, which, precision, D_ip, h, x):
        return nlth_apply_operator(self.h, mesh_h, prob, which, precision, D_ip, h, x)

    def response_spectra(self, vel, dt, periods, h=0.05, kind=0):
        return nlth_response_spectra(self.h, vel, dt, periods, h, kind)

    # -- continuous-batching request loop
    def submit(self, mesh_h, mesh, prob):
        """Queue a solve; returns (ticket, result dict filled on completion)."""
        keep = []
        p = _problem_struct(prob, keep)
        out, res = _result_buffers(p.n_members, p.n_steps, int(np.asarray(mesh.recv).size))
        t = C.c_uint64()
        _check(lib().nlth_submit(self.h, mesh_h, C.byref(p), C.byref(res), C.byref(t)), self.h)
        self._pending = getattr(self, "_pending", {})
        self._pending[t.value] = (keep, res, out)
        return t.value, out

    def poll(self, ticket):
        done = C.c_int32()
        rc = lib().nlth_poll(self.h, C.c_uint64(ticket), C.byref(done))
        return bool(done.value), rc

    def wait(self, ticket, timeout_s=-1.0):
        return lib().nlth_wait(self.h, C.c_uint64(ticket), float(timeout_s))

    def cancel(self, ticket):
        return lib().nlth_cancel(self.h, C.c_uint64(ticket))

    def release(self, ticket):
        """Forget a finished request; its result dict stays valid."""
        rc = lib().nlth_release(self.h, C.c_uint64(ticket))
        if rc == NLTH_OK:
            getattr(self, "_pending", {}).pop(ticket, None)
        return rc

    def close(self):
        for mh in self._meshes:
            lib().nlth_mesh_destroy(mh)
        self._meshes = []
        if self.h:
            lib().nlth_ctx_destroy(self.h)
            self.h = None
