"""Pins for the CPU oracle: closed forms, invariants, textbook values and
independent solvers that a plausible mistake in the oracle would break.

Each test names the passage of arXiv 2604.02755 it checks.  None of the
expected values comes from the HIP path.
"""
import math

import numpy as np
import pytest

from paper_2604_02755_amd import inputs as I


def _iso(lam, mu):
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def _rand_tet(rng):
    while True:
        X = rng.normal(size=(4, 3))
        if np.linalg.det(np.array([X[1] - X[0], X[2] - X[0], X[3] - X[0]])) > 0.05:
            return X


# ---------------------------------------------------------------- geometry

def test_volumes_sum_to_box(oracle_lib):
    """Second-order tets (Section 2.1): element volumes tile the box exactly."""
    for mesh, vol in ((I.box_mesh(4, 3, 2, 1.0), 24.0),
                      (I.perturbed_three_layer_mesh(8, 8, 8, seed=3, amp=0.8, corr=4.0), 512.0)):
        geo = [oracle_lib.tet_geometry(mesh.xyz[t[:4]]) for t in mesh.tet10]
        assert all(g[2] == 0 and g[1] > 0 for g in geo)  # every tet positively oriented
        tot = sum(g[1] for g in geo)
        assert abs(tot - vol) < 1e-11 * vol


def test_barycentric_gradients_reproduce_linear_fields(oracle_lib):
    rng = np.random.default_rng(1)
    X = _rand_tet(rng)
    gL, V, rc = oracle_lib.tet_geometry(X)
    assert rc == 0
    # sum_i x_i (grad L_i)^T = I  (linear precision) and sum grad L_i = 0
    assert np.allclose(X.T @ gL, np.eye(3), atol=1e-12)
    assert np.allclose(gL.sum(0), 0, atol=1e-12)
    assert abs(V - np.linalg.det(np.array([X[1] - X[0], X[2] - X[0], X[3] - X[0]])) / 6) < 1e-14


def test_consistent_mass_matches_textbook_p2_tet(oracle_lib):
    """Consistent mass of the 10-node tet: the textbook V/420 pattern
    (corner diag 6, corner-corner 1, corner-adjacent edge -4, corner-opposite
    edge -6, edge diag 32, edges sharing a vertex 16, opposite edges 8)."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    _, Me = oracle_lib.element_matrices(X, np.zeros((6, 6)), 1.0)
    V = 1 / 6
    Mref = Me[0::3, 0::3] / V  # one component
    edges = I.EDGES
    T = np.zeros((10, 10))
    for a in range(10):
        for b in range(10):
            if a < 4 and b < 4:
                T[a, b] = 6 if a == b else 1
            elif a < 4 or b < 4:
                c, e = (a, b - 4) if a < 4 else (b, a - 4)
                T[a, b] = -4 if c in edges[e] else -6
            else:
                ea, eb = set(edges[a - 4]), set(edges[b - 4])
                T[a, b] = 32 if a == b else (16 if ea & eb else 8)
    assert np.allclose(Mref, T / 420, atol=1e-15)
    # components decouple, total mass rho V per component
    assert abs(Me[0::3, 0::3].sum() - V) < 1e-15
    assert np.allclose(Me[0::3, 1::3], 0)


def test_face_mass_p2_triangle(oracle_lib):
    """6-node triangle int N_a N_b dA: textbook A/180 pattern (corner diag 6,
    corner-corner -1, corner-opposite edge -4, corner-adjacent edge 0, edge
    diag 32, edge-edge 16)."""
    X = np.array([[0, 0, 0], [2, 0, 0], [0, 1, 0.0]])
    M, n, A = oracle_lib.face_matrix(X)
    assert abs(A - 1.0) < 1e-15 and np.allclose(np.abs(n), [0, 0, 1])
    fe = ((0, 1), (1, 2), (2, 0))
    T = np.zeros((6, 6))
    for a in range(6):
        for b in range(6):
            if a < 3 and b < 3:
                T[a, b] = 6 if a == b else -1
            elif a < 3 or b < 3:
                c, e = (a, b - 3) if a < 3 else (b, a - 3)
                T[a, b] = 0 if c in fe[e] else -4
            else:
                T[a, b] = 32 if a == b else 16
    assert np.allclose(M, T * A / 180, atol=1e-15)


# ---------------------------------------------------------------- stiffness

def test_stiffness_symmetric_and_rigid_modes_in_null_space(oracle_lib):
    """Eq. 2 with symmetric D: K_e symmetric, rigid translations and
    rotations produce no force."""
    rng = np.random.default_rng(2)
    X = _rand_tet(rng)
    L = rng.normal(size=(4, 6, 6))
    D = np.einsum("jab,jcb->jac", L, L) + 3 * np.eye(6)
    Ke, _ = oracle_lib.element_matrices(X, D, 1.0)
    assert np.allclose(Ke, Ke.T, rtol=0, atol=1e-12 * np.abs(Ke).max())
    Xn = np.vstack([X, [(X[a] + X[b]) / 2 for a, b in I.EDGES]])
    modes = []
    for c in range(3):
        u = np.zeros((10, 3)); u[:, c] = 1; modes.append(u.ravel())
    for ax in np.eye(3):
        modes.append(np.cross(ax, Xn).ravel())
    for u in modes:
        assert np.abs(Ke @ u).max() <= 1e-13 * np.abs(Ke).max() * np.abs(u).max()
    # positive definite on the complement of the 6 rigid modes
    w = np.linalg.eigvalsh(Ke)
    assert np.sum(w > 1e-10 * w.max()) == 24


def test_element_energy_of_linear_field_is_exact(oracle_lib):
    """Constant strain eps: u^T K_e u = V eps^T D eps (the 4-point rule is exact
    for this; a wrong weight, sign or B entry breaks it)."""
    rng = np.random.default_rng(3)
    X = _rand_tet(rng)
    Xn = np.vstack([X, [(X[a] + X[b]) / 2 for a, b in I.EDGES]])
    F = rng.normal(size=(3, 3))
    u = (Xn @ F.T).ravel()  # u_c = F[c, d] x_d
    eps = np.array([F[0, 0], F[1, 1], F[2, 2], F[0, 1] + F[1, 0], F[1, 2] + F[2, 1], F[2, 0] + F[0, 2]])
    D = _iso(2.0, 1.3)
    Ke, _ = oracle_lib.element_matrices(X, D, 1.0)
    V = oracle_lib.tet_geometry(X)[1]
    assert abs(u @ Ke @ u - V * eps @ D @ eps) < 1e-12 * abs(V * eps @ D @ eps)


def _conical_rule(X, n=4):
    """Points and weights of a conical product Gauss rule on the tet X (4x3):
    the unit cube (a, b, c) maps onto the simplex by xi1 = a, xi2 = b (1 - a),
    xi3 = c (1 - a)(1 - b), with Jacobian 6V (1 - a)^2 (1 - b); Gauss-Legendre
    in each direction (exact here for polynomials of degree 2 n - 3 in x)."""
    g, w = np.polynomial.legendre.leggauss(n)
    g, w = (g + 1) / 2, w / 2
    E = np.array([X[1] - X[0], X[2] - X[0], X[3] - X[0]])
    V6 = abs(np.linalg.det(E))
    pts, wts = [], []
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            for c, wc in zip(g, w):
                xi = np.array([a, b * (1 - a), c * (1 - a) * (1 - b)])
                pts.append(X[0] + xi @ E)
                wts.append(wa * wb * wc * V6 * (1 - a) ** 2 * (1 - b))
    return np.array(pts), np.array(wts)


def test_element_energy_of_quadratic_field_is_exact(oracle_lib):
    """Eq. 2 with the 4-point rule on a quadratic displacement field: the strain
    is linear in x, so eps^T D eps is a quadratic that a rule of degree 2
    integrates exactly.  u^T K_e u must equal the integral taken by an
    independent conical product Gauss rule.  Linear fields cannot tell where the
    four points lie (any points with barycentrics summing to one integrate a
    constant); a quadratic field pins their location (a, b, b, b)."""
    rng = np.random.default_rng(31)
    X = _rand_tet(rng)
    Xn = np.vstack([X, [(X[a] + X[b]) / 2 for a, b in I.EDGES]])
    F = rng.normal(size=(3, 3))
    H = rng.normal(size=(3, 3, 3))
    H = H + H.transpose(0, 2, 1)  # u_c = F[c] . x + x^T H[c] x / 2

    def grad_u(x):  # G[c, d] = d u_c / d x_d
        return F + np.einsum("cde,e->cd", H, x)

    u = np.array([F @ x + 0.5 * np.einsum("cde,d,e->c", H, x, x) for x in Xn]).ravel()
    L = rng.normal(size=(6, 6))
    D = L @ L.T + 2 * np.eye(6)
    Ke, _ = oracle_lib.element_matrices(X, D, 1.0)
    pts, wts = _conical_rule(X)
    energy = 0.0
    for x, wq in zip(pts, wts):
        G = grad_u(x)
        eps = np.array([G[0, 0], G[1, 1], G[2, 2], G[0, 1] + G[1, 0], G[1, 2] + G[2, 1], G[2, 0] + G[0, 2]])
        energy += wq * eps @ D @ eps
    V = oracle_lib.tet_geometry(X)[1]
    assert abs(wts.sum() - V) < 1e-14 * V  # the check rule itself
    assert abs(u @ Ke @ u - energy) < 1e-12 * abs(energy)
    # the field is genuinely quadratic: the centroid strain alone misses the energy
    xc = X.mean(axis=0)
    Gc = grad_u(xc)
    ec = np.array([Gc[0, 0], Gc[1, 1], Gc[2, 2], Gc[0, 1] + Gc[1, 0], Gc[1, 2] + Gc[2, 1], Gc[2, 0] + Gc[0, 2]])
    assert abs(V * ec @ D @ ec - energy) > 1e-3 * abs(energy)


def test_patch_test_on_distorted_mesh(oracle_lib):
    """A linear displacement field on an assembled (distorted) mesh gives zero
    residual at interior nodes."""
    mesh = I.perturbed_three_layer_mesh(4, 4, 4, seed=7, amp=0.3, corr=2.0)
    nn = mesh.n_nodes
    K = np.zeros((3 * nn, 3 * nn))
    D = _iso(5.0, 2.0)
    for t in mesh.tet10:
        Ke, _ = oracle_lib.element_matrices(mesh.xyz[t[:4]], D, 1.0)
        d = (3 * t[:, None] + np.arange(3)).ravel()
        K[np.ix_(d, d)] += Ke
    F = np.array([[1e-3, 2e-3, -1e-3], [0.5e-3, -2e-3, 1e-3], [3e-3, 1e-3, 2e-3]])
    u = (mesh.xyz @ F.T).ravel()
    f = (K @ u).reshape(nn, 3)
    x = mesh.xyz
    interior = ((x[:, 0] > 1e-9) & (x[:, 0] < 4 - 1e-9) & (x[:, 1] > 1e-9) & (x[:, 1] < 4 - 1e-9)
                & (x[:, 2] > -4 + 1e-9) & (x[:, 2] < -1e-9))
    assert interior.sum() > 100
    assert np.abs(f[interior]).max() < 1e-12 * np.abs(f).max()


# ---------------------------------------------------------------- springs

@pytest.mark.parametrize("ns", [12, 150])
def test_spring_table_isotropic(oracle_lib, ns):
    """Multi-spring model (Section 2.1): in the small-strain limit the spring
    sum plus the elastic volumetric part is isotropic elasticity with the
    layer's G0 and bulk modulus; 150 springs per point as in the paper."""
    dirs, w = I.spring_table(ns)
    assert dirs.shape == (ns, 6)
    G0, nu = 1700 * 150.0 ** 2, 0.45
    lam = 2 * G0 * nu / (1 - 2 * nu)
    Kb = lam + 2 * G0 / 3
    D, h = oracle_lib.ip_law(None, None, dirs, w, G0, Kb, 1e-3, 0.2)
    assert np.abs(D - _iso(lam, G0)).max() < 1e-14 * (lam + 2 * G0)
    assert h == 0.0


def test_skeleton_closed_forms(oracle_lib):
    """Modified Ramberg-Osgood skeleton: beta from h_max, secant G/G0 = 1/2 at
    gamma_ref, inverse residual at machine precision, odd symmetry."""
    b = oracle_lib.ro_beta(0.2)
    assert abs(b - 2 * math.pi * 0.2 / (2 - math.pi * 0.2)) < 1e-15
    assert abs(b - 0.9161289188) < 1e-10
    assert abs(oracle_lib.ro_inverse(1.0, b) - 0.5) < 1e-15
    for e in (1e-9, 1e-4, 0.3, 1.0, 7.0, 1e3, 1e6):
        s = oracle_lib.ro_inverse(e, b)
        assert abs(s * (1 + abs(2 * s) ** b) - e) <= 4e-16 * e
        assert oracle_lib.ro_inverse(-e, b) == -s


def _cycle(oracle_lib, amp, n_per_quarter, n_cycles, G0, gref, hmax):
    st = oracle_lib.new_spring()
    g_hist, t_hist = [0.0], [0.0]
    g = 0.0
    path = np.concatenate([np.linspace(0, amp, n_per_quarter + 1)[1:]] +
                          [np.linspace(amp, -amp, 2 * n_per_quarter + 1)[1:],
                           np.linspace(-amp, amp, 2 * n_per_quarter + 1)[1:]] * n_cycles)
    out = []
    for gn in path:
        tau, Gt, hk = oracle_lib.spring_step(st, gn - g, G0, gref, hmax)
        g = gn
        g_hist.append(g)
        t_hist.append(tau)
        out.append((Gt, hk))
    return np.array(g_hist), np.array(t_hist), st, out


@pytest.mark.parametrize("amp_ratio", [0.3, 1.0, 4.0])
def test_masing_loop_closed_form_damping(oracle_lib, amp_ratio):
    """Masing rule on the RO skeleton: the steady loop has tips at +-S(gamma_a)
    and its area gives h = h_max (1 - G_sec/G0), which is also the spring's
    reported equivalent damping."""
    G0, gref, hmax = 4.0e7, 1e-3, 0.2
    amp = amp_ratio * gref
    nq = 4000
    g, t, st, out = _cycle(oracle_lib, amp, nq, 2, G0, gref, hmax)
    b = oracle_lib.ro_beta(hmax)
    S = G0 * gref * oracle_lib.ro_inverse(amp / gref, b)
    # tips
    assert abs(t[nq] - S) < 1e-12 * S
    assert abs(t[3 * nq] + S) < 1e-11 * S
    assert abs(t[-1] - S) < 1e-11 * S
    # area of the last full cycle (trapezoid)
    gl, tl = g[-4 * nq - 1:], t[-4 * nq - 1:]
    area = abs(np.sum(0.5 * (tl[1:] + tl[:-1]) * np.diff(gl)))
    W = 0.5 * S * amp
    h_loop = area / (4 * math.pi * W)
    Gsec = S / amp
    h_closed = hmax * (1 - Gsec / G0)
    assert abs(h_loop - h_closed) < 2e-6 * max(h_closed, 1e-3)
    assert abs(out[-1][1] - h_closed) < 1e-13
    # rejoin at the tip: back on the skeleton with gm = amp
    assert st[5] == 1.0 and abs(st[3] - amp) < 1e-18


def test_masing_branch_residual_and_tangent(oracle_lib):
    """On an unloading branch: gamma - gamma_r = 2 F((tau - tau_r)/2) with F
    the skeleton's strain function, and G_t equals the branch slope."""
    G0, gref, hmax = 3.0e7, 1e-3, 0.2
    b = oracle_lib.ro_beta(hmax)
    st = oracle_lib.new_spring()
    oracle_lib.spring_step(st, 2.5e-3, G0, gref, hmax)
    gr = st[0]
    taus = []
    for _ in range(10):
        tau, Gt, _ = oracle_lib.spring_step(st, -3e-4, G0, gref, hmax)
        taus.append((st[0], tau, Gt))
    tr = st[2]
    assert abs(st[1] - gr) == 0 and st[5] == 0.0
    for gam, tau, Gt in taus:
        x = (tau - tr) / 2 / (G0 * gref)
        F = gref * x * (1 + abs(2 * x) ** b)
        assert abs((gam - gr) - 2 * F) < 1e-13 * gref
    # the secant slope between two branch points lies between their tangents
    slope = (taus[-1][1] - taus[-2][1]) / (taus[-1][0] - taus[-2][0])
    assert taus[-1][2] < slope < taus[-2][2] or taus[-2][2] < slope < taus[-1][2]


def _skeleton_indep(g, G0, gref, beta):
    """S(gamma) from the skeleton's definition e = s (1 + |2 s|^beta) by
    bracketing root search (no Newton): an independent check of the oracle's
    inversion."""
    from scipy.optimize import brentq
    e = g / gref
    if e == 0.0:
        return 0.0
    a = abs(e)
    s = brentq(lambda x: x * (1 + (2 * x) ** beta) - a, 0.0, a, xtol=1e-300, rtol=1e-15, maxiter=500)
    return math.copysign(G0 * gref * s, e)


def test_masing_reversal_on_a_branch_closed_form(oracle_lib):
    """Masing rule (Section 2.1): load on the skeleton to A, unload to A/2 (a
    branch from (A, S(A))), then reload, which reverses while on that branch.
    In closed form tau(A/2) = S(A) - 2 S(A/4); the reload branch starts there,
    tau = tau(A/2) + 2 S((gamma - A/2)/2), so tau(3A/4) = S(A) - 2 S(A/4) +
    2 S(A/8), and at gamma = A it meets the skeleton again, tau = S(A), where
    the spring rejoins it (S(5A/4) beyond).  Taking the reversal stress from
    the skeleton instead of the branch would give S(A/2) at the second
    reversal and fail.  The tangent on the reload branch is the slope of that
    closed form."""
    G0, gref, hmax = 3.0e7, 2.0 ** -10, 0.2
    b = oracle_lib.ro_beta(hmax)
    A = 2.0 ** -10 * 1.5  # binary fractions: every increment below is exact

    def S(x):
        return _skeleton_indep(x, G0, gref, b)

    st = oracle_lib.new_spring()
    n = 64
    seen = {}
    for target, label in ((A, "A"), (A / 2, "A/2"), (3 * A / 4, "3A/4"), (A, "A again"), (5 * A / 4, "5A/4")):
        d = (target - st[0]) / n
        for _ in range(n):
            tau, Gt, _ = oracle_lib.spring_step(st, d, G0, gref, hmax)
        assert st[0] == target
        seen[label] = (tau, Gt, st.copy())
    SA = S(A)
    tol = 1e-13 * SA
    assert abs(seen["A"][0] - SA) < tol
    t_half = SA - 2 * S(A / 4)
    assert abs(seen["A/2"][0] - t_half) < tol
    assert seen["A/2"][2][5] == 0.0  # on a branch
    t_34 = t_half + 2 * S(A / 8)
    assert abs(seen["3A/4"][0] - t_34) < tol
    st34 = seen["3A/4"][2]
    assert st34[1] == A / 2 and abs(st34[2] - t_half) < tol and st34[5] == 0.0
    # tangent: d/dgamma of t_half + 2 S((gamma - A/2)/2) at 3A/4, i.e. S'(A/8)
    hd = A * 1e-5
    slope = (S(A / 8 + hd) - S(A / 8 - hd)) / (2 * hd)
    assert abs(seen["3A/4"][1] - slope) < 1e-7 * slope
    assert abs(seen["A again"][0] - SA) < tol and seen["A again"][2][5] == 1.0
    assert abs(seen["5A/4"][0] - S(5 * A / 4)) < tol and seen["5A/4"][2][3] == 5 * A / 4


def test_single_spring_ip_equals_spring(oracle_lib):
    """N_s = 1 reduces the point law to the textbook single-spring loop: the
    xy-shear entry of D is the spring tangent."""
    G0, Kb, gref, hmax = 2.0e7, 5.0e7, 1e-3, 0.2
    dirs = np.array([[0, 0, 0, 1.0, 0, 0]])
    w = np.array([1.0])
    st_ip = np.array([[0, 0, 0, 0, 0, 1.0]])
    st_sp = oracle_lib.new_spring()
    for dgam in (4e-4, 8e-4, -5e-4, -1e-3, 2e-4, 1.5e-3):
        D, h = oracle_lib.ip_law(np.array([0, 0, 0, dgam, 0, 0]), st_ip, dirs, w, G0, Kb, gref, hmax)
        _, Gt, hk = oracle_lib.spring_step(st_sp, dgam, G0, gref, hmax)
        assert D[3, 3] == Gt and h == hk
        assert np.allclose(D[:3, :3], Kb)


# ---------------------------------------------------------------- damping

def test_rayleigh_least_squares_fit(oracle_lib):
    """Rayleigh damping (Section 2.1): the coefficients are the least-squares
    fit of a/(4 pi f) + pi b f to a unit damping ratio over [f_lo, f_hi]:
    the residual is orthogonal to both basis functions (checked by quadrature)."""
    from scipy.integrate import quad
    a, b = oracle_lib.rayleigh(0.1, 10.0)
    r = lambda f: a / (4 * math.pi * f) + math.pi * b * f - 1
    g1 = quad(lambda f: r(f) / (4 * math.pi * f), 0.1, 10, limit=200)[0]
    g2 = quad(lambda f: r(f) * math.pi * f, 0.1, 10, limit=200)[0]
    assert abs(g1) < 1e-9 and abs(g2) < 1e-7
    assert abs(a - 4.0819) < 1e-4 and abs(b - 0.044671) < 1e-6


# ---------------------------------------------------------------- driver

def test_cg_matches_dense_direct_solve(oracle_lib):
    """The CRS-PCG driver (Alg. 1) against a dense LU stepper on tiny meshes
    (1x1x1 and 2x2x1 cubes) with the nonlinear law active."""
    for dims in ((1, 1, 1), (2, 2, 1)):
        mesh, prob = I.config(0, n_steps=12, mesh_dims=dims, cg_tol=1e-13)
        prob.input_acc *= 50.0  # drive the springs well into the nonlinear range
        r = oracle_lib.run(mesh, prob, want_du=True)
        vel, du = oracle_lib.dense_stepper(mesh, prob)
        assert oracle_lib.rel_l2(r["du"], du) < 1e-10
        assert oracle_lib.rel_l2(r["vel"], vel) < 1e-10


def test_newmark_conserves_energy_undamped(oracle_lib):
    """Section 2.1 state updates are the trapezoidal rule: for a free, undamped
    linear body the energy v^T M v / 2 + u^T K u / 2 is conserved."""
    mesh = I.box_mesh(2, 2, 2, 1.0)
    mesh.bface6 = mesh.bface6[:0]
    mesh.bface_kind = mesh.bface_kind[:0]
    prob = I.make_problem(1, (200.0,), (1800.0,), n_springs=12, n_steps=60, dt=1e-3,
                          damping_mode=I.DAMPING_NONE, cg_tol=1e-14)
    prob.nonlinear[:] = 0
    rng = np.random.default_rng(5)
    v0 = rng.normal(size=3 * mesh.n_nodes) * 1e-3
    r = oracle_lib.run(mesh, prob, want_state=True, v0=v0)
    nn = mesh.n_nodes
    K = np.zeros((3 * nn, 3 * nn)); M = np.zeros((3 * nn, 3 * nn))
    G0 = 1800 * 200.0 ** 2
    lam = 2 * G0 * 0.45 / 0.1
    for t in mesh.tet10:
        Ke, Me = oracle_lib.element_matrices(mesh.xyz[t[:4]], _iso(lam, G0), 1800.0)
        d = (3 * t[:, None] + np.arange(3)).ravel()
        K[np.ix_(d, d)] += Ke
        M[np.ix_(d, d)] += Me
    E0 = 0.5 * v0 @ M @ v0
    E1 = 0.5 * r["v"] @ M @ r["v"] + 0.5 * r["u"] @ K @ r["u"]
    assert abs(E1 - E0) < 1e-10 * E0
    assert 0.5 * r["u"] @ K @ r["u"] > 1e-3 * E0  # energy really moved into strain


def _periodic_column(nz=8):
    """1x1xnz column with x and y periodic ties (alias map) and only the base
    dashpot: a laterally uniform layered half-space model."""
    mesh = I.box_mesh(1, 1, nz, 1.0, I.two_layer(4.0))
    NX = NY = 3
    ids = np.arange(mesh.n_nodes)
    Ii, Jj, Kk = ids % NX, (ids // NX) % NY, ids // (NX * NY)
    alias = (np.where(Ii == 2, 0, Ii) + NX * (np.where(Jj == 2, 0, Jj) + NY * Kk)).astype(np.int32)
    keep = mesh.bface_kind == 0
    mesh.bface6 = np.ascontiguousarray(mesh.bface6[keep])
    mesh.bface_kind = np.ascontiguousarray(mesh.bface_kind[keep])
    top = ids[(Ii == 0) & (Jj == 0) & (Kk == 2 * nz)]
    mesh.recv = top.astype(np.int32)
    return mesh, alias


def test_layer_over_halfspace_resonance(oracle_lib):
    """Linear limit, 1D soil column (top 4 m Vs 150 rho 1700 on Vs 400 rho 1900):
    the transfer function surface / outcrop (= 2 x incident) peaks at
    f = Vs/4H = 9.375 Hz with height rho2 Vs2 / (rho1 Vs1) = 2.98."""
    mesh, alias = _periodic_column(8)
    n = 4096
    acc = np.zeros((1, n, 3))
    # Hann-windowed band-limited noise with zero net velocity change, so the
    # response decays to rest inside the record and the FFT ratio is exact
    win = np.hanning(n // 2)
    w = I.band_limited_wave(77, n // 2, 1e-3, 0.1, 25.0, peak=1e-6) * win
    w -= win * (w.sum() / win.sum())
    acc[0, : n // 2, 0] = w
    prob = I.make_problem(1, (150.0, 400.0), (1700.0, 1900.0), n_springs=12, n_steps=n,
                          input_acc=acc, cg_tol=1e-12)
    r = oracle_lib.run(mesh, prob, alias=alias)
    vs_ = r["vel"][:, 0, 0]
    vI = np.concatenate([[0.0], np.cumsum(0.5 * 1e-3 * (acc[0, 1:, 0] + acc[0, :-1, 0]))])
    vI = vI + 0.5e-3 * acc[0, 0, 0]
    nfft = 1 << 17
    f = np.fft.rfftfreq(nfft, 1e-3)
    with np.errstate(divide="ignore", invalid="ignore"):
        H = np.abs(np.fft.rfft(vs_, nfft)) / np.abs(np.fft.rfft(2 * vI, nfft))
    band = (f > 4) & (f < 15)
    fpk = f[band][np.argmax(H[band])]
    hpk = H[band].max()
    assert abs(fpk - 9.375) < 0.02 * 9.375, fpk
    assert abs(hpk - 1900 * 400 / (1700 * 150)) < 0.05 * 2.98, hpk
    # and the exact 1D transfer function elsewhere in the band (within 5 %)
    k = 2 * np.pi * f / 150.0
    alpha = 1700 * 150 / (1900 * 400)
    H1d = 1 / np.sqrt(np.cos(k * 4) ** 2 + alpha ** 2 * np.sin(k * 4) ** 2)
    sel = (f > 1) & (f < 14)
    assert np.max(np.abs(H[sel] - H1d[sel]) / H1d[sel]) < 0.05


def test_vmax_is_the_largest_velocity_norm(oracle_lib):
    """Maximum velocity-norm maps (Section 3, Figs. 3-4): at each receiver the
    largest |v| over the run, here against the receiver histories the oracle
    records; a nonlinear run reaches every law event (reversals on the
    skeleton and on Masing branches, rejoins), which the GPU parity runs of
    the same setup inherit."""
    mesh, prob = I.config(0, n_steps=30, mesh_dims=(4, 3, 2), cg_tol=1e-12, n_springs=12)
    prob.input_acc *= 5.0
    r = oracle_lib.run(mesh, prob)
    ref = np.sqrt((r["vel"] ** 2).sum(axis=2)).max(axis=0)
    assert ref.max() > 0 and np.allclose(r["vmax"], ref, rtol=1e-15, atol=0)
    assert all(c > 0 for c in r["law_events"][:3]) and r["law_events"][3] == 0, r["law_events"]
    assert 0 <= r["setup_seconds"] <= r["seconds"]


def test_cg_nonconvergence_is_reported(oracle_lib):
    mesh, prob = I.config(0, n_steps=5, mesh_dims=(2, 2, 1))
    prob.cg_maxit = 2
    with pytest.raises(oracle_lib.OracleError) as ei:
        oracle_lib.run(mesh, prob)
    assert ei.value.code == -5


def test_invalid_mesh_rejected(oracle_lib):
    mesh, prob = I.config(0, n_steps=2, mesh_dims=(1, 1, 1))
    t = mesh.tet10.copy()
    t[0, [1, 2]] = t[0, [2, 1]]  # negative Jacobian (and mid-nodes no longer match)
    mesh.tet10 = t
    with pytest.raises(oracle_lib.OracleError) as ei:
        oracle_lib.run(mesh, prob)
    assert ei.value.code == -1


def _ramped_harmonic(f, V, dt, n_ramp=30, n_total=80):
    """Ground velocity whose acceleration is V 2 pi f env(t) cos(2 pi f t),
    env a raised-cosine ramp over n_ramp forcing periods (a slow start keeps
    the free transient of the oscillator small)."""
    Om = 2 * np.pi * f
    t = np.arange(1, int(n_total / f / dt) + 1) * dt
    env = 0.5 - 0.5 * np.cos(np.pi * np.clip(t / (n_ramp / f), 0, 1))
    return np.cumsum(V * Om * env * np.cos(Om * t)) * dt


def test_response_spectra_closed_forms(oracle_lib):
    """Velocity response spectra (Section 3, h = 0.05): under a slowly ramped
    harmonic ground motion the oscillator settles to the textbook steady
    state, |x| = (a_g / w^2) / sqrt((1 - r^2)^2 + (2 h r)^2) and |x'| = W |x|
    (r = W / w, W the forcing frequency), below, near and above resonance;
    a very stiff oscillator follows the ground acceleration (w^2 max|x| = PGA)
    and a very soft one stays put (max|x'| = PGV); no input gives zero."""
    h, T, dt, V = 0.05, 0.5, 2e-4, 0.3
    w = 2 * np.pi / T
    for f in (0.7, 1.7, 3.1):
        Om = 2 * np.pi * f
        v = _ramped_harmonic(f, V, dt)
        r = Om / w
        X = (V * Om / w ** 2) / np.sqrt((1 - r * r) ** 2 + (2 * h * r) ** 2)
        sv, psv = (oracle_lib.response_spectra(v, dt, [T], h, kind=k)[0, 0] for k in (0, 1))
        assert abs(psv / w / X - 1) < 5e-3, (f, psv / w, X)
        assert abs(sv / (Om * X) - 1) < 5e-3, (f, sv, Om * X)
    rng = np.random.default_rng(5)
    v = np.cumsum(np.convolve(rng.normal(size=4000), np.hanning(200), mode="same")) * 1e-3
    a = np.diff(np.concatenate([[0.0], v])) / 1e-3
    stiff = oracle_lib.response_spectra(v, 1e-3, [0.003], h, kind=1)[0, 0] * (2 * np.pi / 0.003)
    soft = oracle_lib.response_spectra(v, 1e-3, [5000.0], h, kind=0)[0, 0]
    assert abs(stiff / np.abs(a).max() - 1) < 2e-2
    assert abs(soft / np.abs(v).max() - 1) < 1e-3
    assert np.all(oracle_lib.response_spectra(np.zeros((2, 50)), 1e-3, [0.1, 1.0], h) == 0.0)


def test_extrapolated_initial_guess_is_closer(oracle_lib):
    """The study behind the library's initial-guess option (the paper does not
    fix the CG initial guess): on the oracle's increments of a benchmark-like
    member (config-2 layers and wave, 8x8x8 cubes, 1 ms steps), once the wave
    is in, the linear extrapolation 2 du^{n-1} - du^{n-2} is an order of
    magnitude closer to du^n than du^{n-1}, and the quadratic one
    3 du^{n-1} - 3 du^{n-2} + du^{n-3} another order closer."""
    mesh, prob = I.config(2, n_members=1, mesh_dims=(8, 8, 8), n_steps=120, cg_tol=1e-12)
    du = oracle_lib.run(mesh, prob, want_du=True)["du"]
    err = []
    for n in range(60, 120):
        nd = np.linalg.norm(du[n])
        err.append([np.linalg.norm(du[n] - g) / nd for g in
                    (du[n - 1], 2 * du[n - 1] - du[n - 2], 3 * du[n - 1] - 3 * du[n - 2] + du[n - 3])])
    e0, e1, e2 = np.median(np.array(err), axis=0)
    assert e1 < e0 / 10 and e2 < e1 / 5, (e0, e1, e2)


def _mem_path(oracle_lib, depth, targets, G0, gref, hmax, n=64):
    st = oracle_lib.new_spring_mem(depth)
    ev = (__import__("ctypes").c_long * 4)()
    seen = []
    for target in targets:
        d = (target - st[0]) / n
        for _ in range(n):
            tau, Gt, _ = oracle_lib.spring_step_mem(st, depth, d, G0, gref, hmax, ev)
        assert st[0] == target
        seen.append((tau, Gt, st.copy()))
    return seen, tuple(ev)


def test_masing_memory_closes_inner_loops(oracle_lib):
    """Masing's rule for inner loops (the law-fidelity extension): with the
    last three reversal points remembered, the path 0 -> A -> -A/2 -> A/4 ->
    -3A/4 -> -A -> -5A/4 closes the inner loop (-A/2 -> A/4 -> -A/2) and goes
    on along the branch from A: in closed form tau(-A/2) = S(A) - 2S(3A/4),
    tau(A/4) = tau(-A/2) + 2S(3A/8), tau(-3A/4) = S(A) - 2S(7A/8), then the
    skeleton at -A and -5A/4.  With the three-rule law (one point) the branch
    from A/4 goes on instead: tau(-3A/4) = tau(A/4) - 2S(A/2).  Depth 1 is
    the oracle's default spring law step for step, and depth 2 behaves as
    depth 1 (an inner loop needs three points)."""
    G0, gref, hmax = 3.0e7, 2.0 ** -10, 0.2
    b = oracle_lib.ro_beta(hmax)
    A = 2.0 ** -10 * 1.5

    def S(x):
        return _skeleton_indep(x, G0, gref, b)

    path = (A, -A / 2, A / 4, -3 * A / 4, -A, -5 * A / 4)
    seen, ev = _mem_path(oracle_lib, 3, path, G0, gref, hmax)
    tol = 1e-13 * S(A)
    t1 = S(A) - 2 * S(3 * A / 4)
    t2 = t1 + 2 * S(3 * A / 8)
    assert abs(seen[0][0] - S(A)) < tol
    assert abs(seen[1][0] - t1) < tol
    assert abs(seen[2][0] - t2) < tol and seen[2][2][6] == 1  # one older point held
    assert abs(seen[3][0] - (S(A) - 2 * S(7 * A / 8))) < tol
    assert seen[3][2][6] == 0 and seen[3][2][1] == A  # back on the branch from A
    assert abs(seen[4][0] + S(A)) < tol and seen[4][2][5] == 1.0  # rejoin at -A
    assert abs(seen[5][0] - S(-5 * A / 4)) < tol
    assert ev[3] == 1 and ev[2] == 1, ev
    # tangent just after the closure: the slope of the branch from A
    hd = A * 1e-5
    slope = (S(7 * A / 8 + hd) - S(7 * A / 8 - hd)) / (2 * hd)
    assert abs(seen[3][1] - slope) < 1e-7 * slope
    # depth 1 (and 2): the three-rule law, equal to or_spring_step throughout
    for depth in (1, 2):
        s1, e1 = _mem_path(oracle_lib, depth, path, G0, gref, hmax)
        assert abs(s1[3][0] - (t2 - 2 * S(A / 2))) < tol and e1[3] == 0
    ref = oracle_lib.new_spring()
    st = oracle_lib.new_spring_mem(1)
    for target in path:
        for _ in range(64):
            d = (target - ref[0]) / 64
            t_ref = oracle_lib.spring_step(ref, d, G0, gref, hmax)
            t_mem = oracle_lib.spring_step_mem(st, 1, d, G0, gref, hmax)
            assert t_ref == t_mem and np.array_equal(ref, st[:6])


def test_masing_memory_stress_stays_continuous(oracle_lib):
    """With enough memory (64 points, more than the reversals of the path) the
    stress never jumps on a random strain path with many nested reversals:
    |tau(g + dg) - tau(g)| <= G0 |dg| (the tangent lies in (0, G0]), through
    every closed inner loop and rejoin.  The three-rule law (depth 1) jumps
    where a branch started inside an earlier loop reaches the largest strain
    and rejoins the skeleton (here 0 -> A -> -A/2 -> A/4 -> -5A/4), which is
    what the memory removes."""
    G0, gref, hmax = 3.0e7, 1e-3, 0.2
    rng = np.random.default_rng(9)
    depth = 64
    st = oracle_lib.new_spring_mem(depth)
    ev = (__import__("ctypes").c_long * 4)()
    tau_prev, g, amp = 0.0, 0.0, 3e-3
    for _ in range(60):
        target = float(np.clip(g + rng.normal(0, 1.5e-3), -amp, amp))
        n = max(1, int(abs(target - g) / 1e-5))
        for _ in range(n):
            dg = (target - g) / n
            tau, Gt, _ = oracle_lib.spring_step_mem(st, depth, dg, G0, gref, hmax, ev)
            assert abs(tau - tau_prev) <= G0 * abs(dg) * (1 + 1e-9) + 1e-6
            assert 0 < Gt <= G0
            tau_prev, g = tau, st[0]
    assert ev[3] >= 5 and ev[2] >= 1, tuple(ev)
    A = 1.5e-3
    jumps = {}
    for depth in (1, 3):
        st = oracle_lib.new_spring_mem(depth)
        tau_prev, big = 0.0, 0.0
        for target in (A, -A / 2, A / 4, -5 * A / 4):
            for _ in range(200):
                dg = (target - st[0]) / 200
                tau, _, _ = oracle_lib.spring_step_mem(st, depth, dg, G0, gref, hmax)
                big = max(big, abs(tau - tau_prev) / (G0 * abs(dg)))
                tau_prev = tau
        jumps[depth] = big
    assert jumps[3] <= 1.0 + 1e-9 and jumps[1] > 1.5, jumps
