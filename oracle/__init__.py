"""Plain FP64 CPU oracle for arXiv 2604.02755 -- TEST INFRASTRUCTURE ONLY.

The oracle is what the HIP path is checked against.  It shares no code with
that path: the arithmetic is in ``oracle.c`` (plain C, FP64, OpenMP loops),
structured as the paper's all-CPU baseline (Section 2.2, Algorithm 1: per step
assemble 3x3-block CRS from the current D, block-Jacobi PCG for Eq. 1, then the
multi-spring law at every integration point).  This module only marshals
arguments through ctypes and adds :func:`dense_stepper`, a NumPy dense
assembly + LU time stepper used as an independent check of the CRS-PCG driver
on tiny meshes.

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (in place)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"],
                              cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int), ("xyz", _dp), ("n_tets", C.c_int), ("tet10", _ip),
                ("layer", _ip), ("n_bfaces", C.c_int), ("bface6", _ip),
                ("bface_kind", C.POINTER(C.c_ubyte)), ("n_recv", C.c_int), ("recv", _ip),
                ("alias", _ip)]


class _Problem(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("rho", _dp), ("vs", _dp), ("nu", _dp),
                ("gamma_ref", _dp), ("h_max", _dp), ("nonlinear", _ip), ("n_springs", C.c_int),
                ("dirs", _dp), ("weights", _dp), ("damping_mode", C.c_int), ("h0", C.c_double),
                ("f_lo", C.c_double), ("f_hi", C.c_double), ("dt", C.c_double),
                ("n_steps", C.c_int), ("input_acc", _dp), ("cg_tol", C.c_double),
                ("cg_maxit", C.c_int), ("v0", _dp), ("apply_which", C.c_int), ("apply_D", _dp),
                ("apply_h", _dp), ("apply_x", _dp), ("apply_y", _dp), ("masing_depth", C.c_int)]


class _Result(C.Structure):
    _fields_ = [("vel", _dp), ("iters", _ip), ("du_hist", _dp), ("u_final", _dp),
                ("v_final", _dp), ("D_final", _dp), ("h_final", _dp), ("theta_final", _dp), ("vmax", _dp),
                ("law_events", C.c_long * 4), ("setup_seconds", C.c_double), ("steps_done", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB_PATH)
        _lib.or_run.argtypes = [C.POINTER(_Mesh), C.POINTER(_Problem), C.POINTER(_Result)]
        _lib.or_last_error.restype = C.c_char_p
        _lib.or_ro_inverse.restype = C.c_double
        _lib.or_ro_inverse.argtypes = [C.c_double, C.c_double]
        _lib.or_ro_beta.restype = C.c_double
        _lib.or_ro_beta.argtypes = [C.c_double]
        _lib.or_spring_step.restype = C.c_double
        _lib.or_spring_step.argtypes = [_dp, C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp]
        _lib.or_tet_geometry.argtypes = [_dp, _dp, _dp]
        _lib.or_element_matrices.argtypes = [_dp, _dp, C.c_double, _dp, _dp]
        _lib.or_face_matrix.argtypes = [_dp, _dp, _dp, _dp]
        _lib.or_rayleigh.argtypes = [C.c_double, C.c_double, _dp, _dp]
        _lib.or_ip_law.argtypes = [_dp, _dp, C.c_int, _dp, _dp, C.c_double, C.c_double,
                                   C.c_double, C.c_double, _dp, _dp]
        _lib.or_set_threads.argtypes = [C.c_int]
        _lib.or_spring_step_mem.restype = C.c_double
        _lib.or_spring_step_mem.argtypes = [_dp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, _dp,
                                            _dp, C.POINTER(C.c_long)]
        _lib.or_spring_words.restype = C.c_int
        _lib.or_spring_words.argtypes = [C.c_int]
    return _lib


def _p(a, ct=_dp):
    return a.ctypes.data_as(ct) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    def __init__(self, code, msg, partial=None):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code
        self.partial = partial


def run(mesh, prob, member: int = 0, alias=None, want_du: bool = False, want_state: bool = False,
        n_steps: int | None = None, cg_tol: float | None = None, v0=None):
    """Run one member of ``prob`` on ``mesh``.  Returns a dict of numpy arrays.

    ``vel``: [n_steps, n_recv, 3]; ``vmax``: [n_recv], the largest velocity
    norm over the run at each receiver; ``iters``: [n_steps]; ``law_events``:
    counts over the run of (reversals on the skeleton, reversals on a Masing
    branch, rejoins of the skeleton, inner loops closed); optional ``du``
    [n_steps, n_dof]; ``u``, ``D`` [n_tets, 4, 21], ``h`` [n_tets], ``theta``
    [n_tets, 4, n_springs, W] (W = 6 for the three-rule law);
    ``seconds`` wall time, of which ``setup_seconds`` before the first step.
    """
    L = lib()
    keep = []

    def k(a):
        keep.append(a)
        return a

    ns = int(n_steps if n_steps is not None else prob.n_steps)
    xyz = k(_f64(mesh.xyz))
    tet = k(_i32(mesh.tet10))
    lay = k(_i32(mesh.layer))
    bf = k(_i32(mesh.bface6))
    bk = k(np.ascontiguousarray(mesh.bface_kind, dtype=np.uint8))
    rc = k(_i32(mesh.recv))
    al = k(_i32(alias)) if alias is not None else None
    m = _Mesh(mesh.n_nodes, _p(xyz), mesh.n_tets, _p(tet, _ip), _p(lay, _ip), int(bf.shape[0]),
              _p(bf, _ip), bk.ctypes.data_as(C.POINTER(C.c_ubyte)), int(rc.size), _p(rc, _ip),
              _p(al, _ip) if al is not None else None)
    rho, vs, nu, gr = (k(_f64(np.asarray(getattr(prob, f))[member])) for f in ("rho", "vs", "nu", "gamma_ref"))
    hm = k(_f64(prob.h_max))
    nl = k(_i32(prob.nonlinear))
    dirs = k(_f64(prob.dirs))
    w = k(_f64(prob.weights))
    acc = k(_f64(np.asarray(prob.input_acc)[member][:ns]))
    p = _Problem(prob.n_layers, _p(rho), _p(vs), _p(nu), _p(gr), _p(hm), _p(nl, _ip),
                 prob.n_springs, _p(dirs), _p(w), int(prob.damping_mode), float(prob.h0),
                 float(prob.f_lo), float(prob.f_hi), float(prob.dt), ns, _p(acc),
                 float(cg_tol if cg_tol is not None else prob.cg_tol), int(prob.cg_maxit),
                 _p(k(_f64(v0))) if v0 is not None else None, -1, None, None, None, None,
                 int(getattr(prob, "masing_depth", 1) or 1))
    out = dict(vel=np.zeros((ns, rc.size, 3)), iters=np.zeros(ns, np.int32), vmax=np.zeros(rc.size))
    if want_du:
        out["du"] = np.zeros((ns, 3 * mesh.n_nodes))
    if want_state:
        out["u"] = np.zeros(3 * mesh.n_nodes)
        out["v"] = np.zeros(3 * mesh.n_nodes)
        out["D"] = np.zeros((mesh.n_tets, 4, 21))
        out["h"] = np.zeros(mesh.n_tets)
        out["theta"] = np.zeros((mesh.n_tets, 4, prob.n_springs,
                                 L.or_spring_words(int(getattr(prob, "masing_depth", 1) or 1))))
    r = _Result(_p(out["vel"]), _p(out["iters"], _ip), _p(out.get("du")), _p(out.get("u")),
                _p(out.get("v")), _p(out.get("D")), _p(out.get("h")), _p(out.get("theta")), _p(out["vmax"]),
                (C.c_long * 4)(), 0.0, 0)
    t0 = time.perf_counter()
    code = L.or_run(C.byref(m), C.byref(p), C.byref(r))
    out["seconds"] = time.perf_counter() - t0
    out["steps_done"] = r.steps_done
    out["setup_seconds"] = r.setup_seconds
    out["law_events"] = tuple(int(x) for x in r.law_events)
    if code != 0:
        raise OracleError(code, L.or_last_error().decode(), out)
    return out


def set_threads(n: int):
    """Threads of the oracle's OpenMP loops (for timing on a stated core count)."""
    lib().or_set_threads(int(n))


def apply_operator(mesh, prob, which, D_ip, h, x, member: int = 0):
    """y = Op x with the oracle's assembled CRS matrices (Op: 0 A, 1 K, 2 M)."""
    L = lib()
    keep = []

    def k(a):
        keep.append(a)
        return a

    xyz, tet, lay = k(_f64(mesh.xyz)), k(_i32(mesh.tet10)), k(_i32(mesh.layer))
    bf, rc = k(_i32(mesh.bface6)), k(_i32(mesh.recv))
    bk = k(np.ascontiguousarray(mesh.bface_kind, dtype=np.uint8))
    m = _Mesh(mesh.n_nodes, _p(xyz), mesh.n_tets, _p(tet, _ip), _p(lay, _ip), int(bf.shape[0]),
              _p(bf, _ip), bk.ctypes.data_as(C.POINTER(C.c_ubyte)), int(rc.size), _p(rc, _ip), None)
    rho, vs, nu, gr = (k(_f64(np.asarray(getattr(prob, f))[member])) for f in ("rho", "vs", "nu", "gamma_ref"))
    hm, nl, dirs, w = k(_f64(prob.h_max)), k(_i32(prob.nonlinear)), k(_f64(prob.dirs)), k(_f64(prob.weights))
    D = k(_f64(D_ip).reshape(-1))
    hh = k(_f64(h)) if h is not None else None
    xx = k(_f64(x))
    y = np.zeros_like(xx)
    p = _Problem(prob.n_layers, _p(rho), _p(vs), _p(nu), _p(gr), _p(hm), _p(nl, _ip), prob.n_springs,
                 _p(dirs), _p(w), int(prob.damping_mode), float(prob.h0), float(prob.f_lo), float(prob.f_hi),
                 float(prob.dt), 0, None, 1e-8, 1, None, int(which), _p(D), _p(hh), _p(xx), _p(y), 1)
    out = _Result(_p(np.zeros(1)), None, None, None, None, None, None, None, None, (C.c_long * 4)(), 0.0, 0)
    code = L.or_run(C.byref(m), C.byref(p), C.byref(out))
    if code != 0:
        raise OracleError(code, L.or_last_error().decode())
    return y


# ---------------------------------------------------------------------------
# building blocks (for the pins)
# ---------------------------------------------------------------------------

def tet_geometry(X4):
    X = _f64(X4).reshape(12)
    gL = np.zeros(12)
    v = C.c_double()
    rc = lib().or_tet_geometry(_p(X), _p(gL), C.byref(v))
    return gL.reshape(4, 3), v.value, rc


def element_matrices(X4, D4, rho):
    """30x30 stiffness (Eq. 2, 4-point rule) and consistent mass of one tet."""
    X = _f64(X4).reshape(12)
    D = _f64(np.broadcast_to(np.asarray(D4, float).reshape(-1, 6, 6), (4, 6, 6))).reshape(144)
    Ke = np.zeros(900)
    Me = np.zeros(900)
    lib().or_element_matrices(_p(X), _p(D), float(rho), _p(Ke), _p(Me))
    return Ke.reshape(30, 30), Me.reshape(30, 30)


def face_matrix(X3):
    X = _f64(X3).reshape(9)
    M = np.zeros(36)
    n = np.zeros(3)
    a = C.c_double()
    lib().or_face_matrix(_p(X), _p(M), _p(n), C.byref(a))
    return M.reshape(6, 6), n, a.value


def rayleigh(f_lo, f_hi):
    a, b = C.c_double(), C.c_double()
    lib().or_rayleigh(float(f_lo), float(f_hi), C.byref(a), C.byref(b))
    return a.value, b.value


def ro_beta(h_max):
    return lib().or_ro_beta(float(h_max))


def ro_inverse(e, beta):
    return lib().or_ro_inverse(float(e), float(beta))


def new_spring():
    """Virgin spring state: gp, gr, tr, gm = 0, dir = 0, on the skeleton."""
    return np.array([0.0, 0.0, 0.0, 0.0, 0.0, 1.0])


def spring_step(state, dgamma, G0, gref, h_max):
    """Advance one spring by ``dgamma``; returns (tau, G_t, h_k), mutates state."""
    Gt, hk = C.c_double(), C.c_double()
    tau = lib().or_spring_step(_p(state), float(dgamma), float(G0), float(gref), float(h_max),
                               C.byref(Gt), C.byref(hk))
    return tau, Gt.value, hk.value


def new_spring_mem(depth):
    """Virgin spring state with a reversal memory of ``depth`` points."""
    st = np.zeros(lib().or_spring_words(int(depth)))
    st[5] = 1.0
    return st


def spring_step_mem(state, depth, dgamma, G0, gref, h_max, events=None):
    """Advance one spring with a reversal memory of ``depth``; returns
    (tau, G_t, h_k); ``events`` (4 longs) accumulates the law events."""
    Gt, hk = C.c_double(), C.c_double()
    ev = events if events is not None else (C.c_long * 4)()
    tau = lib().or_spring_step_mem(_p(state), int(depth), float(dgamma), float(G0), float(gref), float(h_max),
                                   C.byref(Gt), C.byref(hk), ev)
    return tau, Gt.value, hk.value


def ip_law(deps, state, dirs, weights, G0, Kb, gref, h_max):
    """One integration point of the multi-spring law; returns (D 6x6, h)."""
    D = np.zeros(36)
    h = C.c_double()
    d = _f64(deps) if deps is not None else None
    lib().or_ip_law(_p(d), _p(state), int(dirs.shape[0]), _p(_f64(dirs)), _p(_f64(weights)),
                    float(G0), float(Kb), float(gref), float(h_max), _p(D), C.byref(h))
    return D.reshape(6, 6), h.value


def new_ip_state(n_springs):
    st = np.zeros((n_springs, 6))
    st[:, 5] = 1.0
    return st


# ---------------------------------------------------------------------------
# NumPy dense-direct time stepper (tiny meshes)
# ---------------------------------------------------------------------------

def dense_stepper(mesh, prob, member: int = 0, n_steps: int | None = None):
    """Independent driver for tiny meshes: dense global matrices, LU solves.

    It uses the oracle's element, face and law building blocks but none of its
    CRS, CG or assembly code: K, M and C are assembled densely with numpy,
    Eq. 1 is solved with ``numpy.linalg.solve`` and the state updates of
    Section 2.1 are applied in numpy.  Returns (vel [n_steps, n_recv, 3],
    du [n_steps, n_dof]).
    """
    ns = int(n_steps or prob.n_steps)
    nn, ne = mesh.n_nodes, mesh.n_tets
    ndof = 3 * nn
    dt = prob.dt
    lay = np.asarray(mesh.layer)
    rho = np.asarray(prob.rho)[member]
    vs = np.asarray(prob.vs)[member]
    nu = np.asarray(prob.nu)[member]
    gref = np.asarray(prob.gamma_ref)[member]
    G0 = rho * vs ** 2
    lam = 2 * G0 * nu / (1 - 2 * nu)
    Kb = lam + 2 * G0 / 3
    vp = np.sqrt((lam + 2 * G0) / rho)
    X = mesh.xyz[mesh.tet10[:, :4]]
    dofs = (3 * mesh.tet10[:, :, None] + np.arange(3)).reshape(ne, 30)

    M = np.zeros((ndof, ndof))
    for e in range(ne):
        _, Me = element_matrices(X[e], np.zeros((4, 6, 6)), rho[lay[e]])
        M[np.ix_(dofs[e], dofs[e])] += Me
    # faces
    Cabs = np.zeros((ndof, ndof))
    fbase = np.zeros(ndof * 3).reshape(ndof, 3)
    face_layer = _face_layers(mesh)
    for f in range(mesh.bface6.shape[0]):
        nodes = mesh.bface6[f]
        Mf, n, _ = face_matrix(mesh.xyz[nodes[:3]])
        l = face_layer[f]
        Z = rho[l] * (vp[l] * np.outer(n, n) + vs[l] * (np.eye(3) - np.outer(n, n)))
        fd = (3 * nodes[:, None] + np.arange(3)).ravel()
        Cabs[np.ix_(fd, fd)] += np.kron(Mf, Z)
        if mesh.bface_kind[f] == 0:
            fbase[fd] += np.kron(Mf.sum(axis=1)[:, None], Z)
    ahat, bhat = rayleigh(prob.f_lo, prob.f_hi)

    ip_state = [[new_ip_state(prob.n_springs) for _ in range(4)] for _ in range(ne)]
    D = np.zeros((ne, 4, 6, 6))
    for e in range(ne):
        l = lay[e]
        for j in range(4):
            D[e, j], _ = ip_law(None, None, prob.dirs, prob.weights, G0[l], Kb[l], gref[l], prob.h_max[l])
    h = np.zeros(ne)
    u = np.zeros(ndof); v = np.zeros(ndof); a = np.zeros(ndof); q = np.zeros(ndof)
    vI = np.zeros(3); aprev = np.zeros(3)
    vel = np.zeros((ns, mesh.recv.size, 3))
    dus = np.zeros((ns, ndof))
    # B matrices at the 4 points (for the strain increments)
    QA, QB = 0.5854101966249685, 0.1381966011250105
    edges = ((0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3))
    for n in range(1, ns + 1):
        an = np.asarray(prob.input_acc)[member, n - 1]
        vI = vI + 0.5 * dt * (aprev + an)
        aprev = an
        K = np.zeros((ndof, ndof))
        C_ = Cabs.copy()
        for e in range(ne):
            Ke, Me = element_matrices(X[e], D[e], rho[lay[e]])
            hh = h[e] if prob.damping_mode == 0 else (prob.h0 if prob.damping_mode == 1 else 0.0)
            ix = np.ix_(dofs[e], dofs[e])
            K[ix] += Ke
            C_[ix] += ahat * hh * Me + bhat * hh * Ke
        A = 4 / dt ** 2 * M + 2 / dt * C_ + K
        f = 2 * fbase @ vI
        b = f - q + C_ @ v + M @ (a + 4 / dt * v)
        du = np.linalg.solve(A, b)
        q = q + K @ du
        u = u + du
        a = -a - 4 / dt * v + 4 / dt ** 2 * du
        v = -v + 2 / dt * du
        for e in range(ne):
            l = lay[e]
            if not prob.nonlinear[l]:
                h[e] = 0.0
                continue
            gL, _, _ = tet_geometry(X[e])
            due = du[dofs[e]].reshape(10, 3)
            hs = 0.0
            for j in range(4):
                Lb = np.full(4, QB); Lb[j] = QA
                G = np.zeros((10, 3))
                for i in range(4):
                    G[i] = (4 * Lb[i] - 1) * gL[i]
                for k_, (p_, q_) in enumerate(edges):
                    G[4 + k_] = 4 * (Lb[p_] * gL[q_] + Lb[q_] * gL[p_])
                F = due.T @ G  # F[c, d] = d u_c / d x_d
                de = np.array([F[0, 0], F[1, 1], F[2, 2], F[0, 1] + F[1, 0], F[1, 2] + F[2, 1],
                               F[2, 0] + F[0, 2]])
                D[e, j], hj = ip_law(de, ip_state[e][j], prob.dirs, prob.weights, G0[l], Kb[l],
                                     gref[l], prob.h_max[l])
                hs += hj
            h[e] = hs / 4
        vel[n - 1] = v.reshape(nn, 3)[mesh.recv]
        dus[n - 1] = du
    return vel, dus


def _face_layers(mesh):
    """Layer of the tet that owns each boundary face."""
    faces = {}
    for e in range(mesh.n_tets):
        t = mesh.tet10[e]
        for tri in ((0, 1, 2), (1, 2, 3), (0, 2, 3), (0, 1, 3)):
            faces[tuple(sorted(int(t[i]) for i in tri))] = e
    return np.array([mesh.layer[faces[tuple(sorted(int(x) for x in f[:3]))]] for f in mesh.bface6])


def rel_l2(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


# ---------------------------------------------------------------------------
# velocity response spectra of receiver records (Section 3: the surface
# waveforms are compared through velocity response spectra with h = 0.05)
# ---------------------------------------------------------------------------

def response_spectra(vel, dt, periods, h=0.05, kind=0):
    """Response spectra of ground-velocity records.

    vel: [n_series, n_steps] samples v_1..v_N at t_n = n dt, with v_0 = 0.
    The velocity is taken linear between samples, so the ground acceleration
    is constant on each step, a_n = (v_n - v_{n-1}) / dt.  The oscillator
    x'' + 2 h w x' + w^2 x = -a_g (w = 2 pi / T, x relative to the ground)
    starts at rest and is advanced exactly over each step: the state
    (x, x', a) evolves under a constant augmented matrix, so one step is the
    matrix exponential of that matrix times dt (a library routine).
    kind 0: relative velocity spectrum max_n |x'_n|; kind 1: pseudo-velocity
    w max_n |x_n|.  Returns [n_series, n_periods]."""
    from scipy.linalg import expm
    v = np.asarray(vel, dtype=np.float64)
    v = v.reshape(1, -1) if v.ndim == 1 else v
    ns, nt = v.shape
    a = np.diff(np.concatenate([np.zeros((ns, 1)), v], axis=1), axis=1) / dt
    out = np.zeros((ns, len(periods)))
    for k, T in enumerate(periods):
        w = 2.0 * np.pi / T
        Maug = np.array([[0.0, 1.0, 0.0], [-w * w, -2.0 * h * w, -1.0], [0.0, 0.0, 0.0]])
        E = expm(Maug * dt)
        Phi, Gam = E[:2, :2], E[:2, 2]
        x = np.zeros((2, ns))
        peak_x = np.zeros(ns)
        peak_v = np.zeros(ns)
        for n in range(nt):
            x = Phi @ x + np.outer(Gam, a[:, n])
            peak_x = np.maximum(peak_x, np.abs(x[0]))
            peak_v = np.maximum(peak_v, np.abs(x[1]))
        out[:, k] = peak_v if kind == 0 else w * peak_x
    return out
