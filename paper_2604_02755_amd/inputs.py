"""Seeded synthetic inputs for the nonlinear time-history ensemble solver.

This module is the only code shared by the HIP path and the CPU oracle, and it
holds none of the method's arithmetic: it produces the *data* a problem is made
of -- a second-order tetrahedral box mesh with its absorbing-boundary faces and
receivers, the multi-spring direction table, per-member layer properties and
band-limited incident base accelerations.  Nothing here evaluates shape
functions, element matrices, the spring law, the solver or time stepping.

Workload recipe (the paper's Tokyo model, Section 2.3, is not available, so
these seeded boxes stand in for it):

* Box of ``nx*ny*nz`` cubes of edge ``h``; each cube is split into the six
  Kuhn tetrahedra sharing its main diagonal; every tet is a 10-node quadratic
  tetrahedron (Section 2.1: second-order tets are used for strain evaluation)
  whose mid-edge nodes sit at the exact edge midpoints, so the node set is
  the full half-step lattice.
* Node order follows VTK's quadratic tetra: v0..v3, then the edges
  01, 12, 20, 03, 13, 23.
* Free surface at z = 0, base at z = -nz*h.  Base faces (kind 0) carry the
  absorbing dashpot and the incident wave; side faces (kind 1) are absorbing
  (Section 2.1: absorbing boundaries on the bottom and sides).
* Multi-spring directions (Section 2.1, multi-spring model with 150 springs per
  material point): plane normals on icosahedral axes, slip directions in the
  plane; the orbit is a spherical 5-design, which makes the spring sum exactly
  isotropic in the small-strain limit.
* Incident base accelerations: white Gaussian noise, band-limited by zeroing
  FFT bins outside [f_lo, f_hi], ramped in and scaled to a peak per component
  (x and y twice z, the paper's 0.6 : 0.3 ratio in Section 2.3).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# VTK quadratic-tetra edge list: node 4+i is the midpoint of EDGES[i].
EDGES = ((0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3))
# Faces of a tet as vertex triples (the face opposite vertex 3, 0, 1, 2).
FACES = ((0, 1, 2), (1, 2, 3), (0, 2, 3), (0, 1, 3))

DAMPING_LAW, DAMPING_CONST, DAMPING_NONE = 0, 1, 2
PRECISION_FP64, PRECISION_MIXED = 0, 1


@dataclass
class Mesh:
    """Tet10 mesh arrays (all numpy, C-contiguous)."""

    xyz: np.ndarray          # float64 [n_nodes, 3]
    tet10: np.ndarray        # int32 [n_tets, 10], VTK quadratic-tetra order
    layer: np.ndarray        # int32 [n_tets]
    bface6: np.ndarray       # int32 [n_bfaces, 6]: 3 vertices then midpoints of (ab, bc, ca)
    bface_kind: np.ndarray   # uint8 [n_bfaces]: 0 base (absorbing + input), 1 side
    recv: np.ndarray         # int32 [n_recv] receiver nodes
    dims: tuple = (0, 0, 0)
    surface: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tet10.shape[0])

    @property
    def n_dof(self) -> int:
        return 3 * self.n_nodes


def _lattice_id(I, J, K, NX, NY):
    return I + NX * (J + NY * K)


def box_mesh(nx: int, ny: int, nz: int, h: float = 1.0, layer_of_depth=None,
             recv_stride: int = 1) -> Mesh:
    """Kuhn-split box of ``nx*ny*nz`` cubes of edge ``h`` as quadratic tets.

    ``layer_of_depth(depth_of_cube_centre) -> int`` assigns the layer id
    (default: everything layer 0).  Receivers are every ``recv_stride``-th
    surface lattice node in x and y (stride 1: all surface nodes).
    """
    NX, NY, NZ = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    I, J, K = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    ids = _lattice_id(I, J, K, NX, NY)
    xyz = np.zeros((NX * NY * NZ, 3))
    xyz[ids.ravel(), 0] = I.ravel() * (h / 2)
    xyz[ids.ravel(), 1] = J.ravel() * (h / 2)
    xyz[ids.ravel(), 2] = -nz * h + K.ravel() * (h / 2)

    # Six Kuhn tets per cube, one per axis permutation (lexicographic order);
    # corners in doubled lattice units relative to the cube origin.
    local = []
    for perm in itertools.permutations(range(3)):
        v = [np.zeros(3, int)]
        for ax in perm:
            nv = v[-1].copy()
            nv[ax] += 2
            v.append(nv)
        v0, v1, v2, v3 = v
        if np.linalg.det(np.array([v1 - v0, v2 - v0, v3 - v0], float)) < 0:
            v1, v2 = v2, v1
        verts = [v0, v1, v2, v3]
        nodes = verts + [(verts[a] + verts[b]) // 2 for a, b in EDGES]
        local.append(np.array(nodes))
    local = np.array(local)  # [6, 10, 3] doubled-lattice offsets

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # cube order: i fastest, then j, then k
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    nc = ci.size
    LI = 2 * ci[:, None, None] + local[None, :, :, 0]
    LJ = 2 * cj[:, None, None] + local[None, :, :, 1]
    LK = 2 * ck[:, None, None] + local[None, :, :, 2]
    tet10 = _lattice_id(LI, LJ, LK, NX, NY).reshape(nc * 6, 10).astype(np.int32)

    depth = (nz - ck - 0.5) * h
    if layer_of_depth is None:
        layer_c = np.zeros(nc, np.int32)
    else:
        layer_c = np.array([layer_of_depth(d) for d in depth], np.int32)
    layer = np.repeat(layer_c, 6).astype(np.int32)

    # Boundary faces: a tet face all of whose vertices lie on one outer plane.
    LI4, LJ4, LK4 = LI.reshape(-1, 10), LJ.reshape(-1, 10), LK.reshape(-1, 10)
    bf, kind = [], []
    planes = ((LK4, 0, 0), (LI4, 0, 1), (LI4, NX - 1, 1), (LJ4, 0, 1), (LJ4, NY - 1, 1))
    for a, b, c in FACES:
        mids = [_edge_index(a, b), _edge_index(b, c), _edge_index(c, a)]
        cols = [a, b, c] + [4 + m for m in mids]
        for arr, val, kd in planes:
            on = (arr[:, a] == val) & (arr[:, b] == val) & (arr[:, c] == val)
            if on.any():
                bf.append(tet10[on][:, cols])
                kind.append(np.full(int(on.sum()), kd, np.uint8))
    bface6 = np.ascontiguousarray(np.concatenate(bf).astype(np.int32))
    bface_kind = np.ascontiguousarray(np.concatenate(kind))

    surf = np.sort(ids[:, :, NZ - 1].ravel()).astype(np.int32)
    recv = np.sort(ids[::recv_stride, ::recv_stride, NZ - 1].ravel()).astype(np.int32)
    return Mesh(xyz=np.ascontiguousarray(xyz), tet10=np.ascontiguousarray(tet10),
                layer=layer, bface6=bface6, bface_kind=bface_kind,
                recv=np.ascontiguousarray(recv), dims=(nx, ny, nz), surface=surf)


def _edge_index(a: int, b: int) -> int:
    for i, (p, q) in enumerate(EDGES):
        if (p, q) == (a, b) or (q, p) == (a, b):
            return i
    raise ValueError((a, b))


def two_layer(top_depth: float = 4.0):
    """Layer id by cube-centre depth: 0 above ``top_depth``, 1 below."""
    return lambda d: 0 if d < top_depth else 1


def smooth_field(n: int, seed: int, corr: float, amp: float, spacing: float = 1.0) -> np.ndarray:
    """Seeded smooth random surface on an n x n vertex grid.

    White N(0,1) convolved (periodically, via FFT) with exp(-2 r^2 / corr^2),
    whose autocorrelation is exp(-r^2 / corr^2); scaled to max |.| = amp.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    r = np.minimum(np.arange(n), n - np.arange(n)) * spacing
    g1 = np.exp(-2.0 * r ** 2 / corr ** 2)
    g = np.outer(g1, g1)
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * np.fft.fft2(g)))
    return f * (amp / np.max(np.abs(f)))


def perturbed_three_layer_mesh(nx: int, ny: int, nz: int, seed: int, amp: float = 3.0,
                               corr: float = 30.0, recv_stride: int = 4) -> Mesh:
    """Three layers with interfaces perturbed by seeded smooth random surfaces.

    Vertex levels (counted from the base) ``3nz/4`` and ``3nz/8``... are
    snapped to their mean height plus an independent smooth field of
    amplitude ``amp`` and correlation ``corr``; intermediate vertex levels are
    re-spaced linearly per column; top and base stay flat; mid-edge nodes are
    reset to the midpoints so every tet stays straight-sided.  The layer id is
    the cube's original band: top (0) above the upper interface, middle (1),
    bottom (2).
    """
    m = box_mesh(nx, ny, nz, 1.0, None, recv_stride)
    NX, NY, NZ = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    k_up, k_lo = (3 * nz) // 4, (3 * nz) // 8   # 24 and 12 for nz = 32
    z0 = -float(nz)
    f_up = smooth_field(max(NX, NY) // 2 + 1, seed, corr, amp)[: nx + 1, : ny + 1]
    f_lo = smooth_field(max(NX, NY) // 2 + 1, seed + 1, corr, amp)[: nx + 1, : ny + 1]
    # vertex-level heights per column
    kv = np.arange(nz + 1, dtype=float)
    zc = np.empty((nx + 1, ny + 1, nz + 1))
    fixed_k = [0, k_lo, k_up, nz]
    for ix in range(nx + 1):
        for iy in range(ny + 1):
            fixed_z = [z0, z0 + k_lo + f_lo[ix, iy], z0 + k_up + f_up[ix, iy], 0.0]
            zc[ix, iy] = np.interp(kv, fixed_k, fixed_z)
    xyz = m.xyz.copy()
    I, J, K = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    ids = _lattice_id(I, J, K, NX, NY)
    # vertices: all-even lattice indices; others: averages of the two (or more)
    # vertex endpoints of the edge they are the midpoint of.  Because each
    # half-lattice point is the midpoint of its containing edge, its height is
    # the mean of the heights at floor/ceil lattice corners along odd axes.
    zv = zc  # [nx+1, ny+1, nz+1]
    Ie, Je, Ke = I // 2, J // 2, K // 2
    Io, Jo, Ko = I % 2, J % 2, K % 2
    # the midpoint of an edge (vertex A, vertex B) where the odd axes step by +1
    # in each odd direction: the Kuhn edges are along (1,0,0),(1,1,0),(1,1,1)
    # type directions, all with non-negative steps, so A = floor, B = ceil.
    zA = zv[Ie, Je, Ke]
    zB = zv[Ie + Io, Je + Jo, Ke + Ko]
    xyz[ids.ravel(), 2] = (0.5 * (zA + zB)).ravel()
    def lay(ck):
        return 0 if ck >= k_up else (1 if ck >= k_lo else 2)
    nc = nx * ny * nz
    ck = np.arange(nc) // (nx * ny)
    layer = np.repeat(np.array([lay(c) for c in ck], np.int32), 6)
    m.xyz = np.ascontiguousarray(xyz)
    m.layer = layer
    return m


# --------------------------------------------------------------------------
# Multi-spring direction table (Section 2.1, multi-spring model)
# --------------------------------------------------------------------------

def _icosahedron_vertices() -> np.ndarray:
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for s1 in (1.0, -1.0):
        for s2 in (1.0, -1.0):
            v += [(0.0, s1, s2 * phi), (s1, s2 * phi, 0.0), (s2 * phi, 0.0, s1)]
    v = np.array(v)
    return v / np.linalg.norm(v, axis=1)[:, None]


def _merge_antipodes(p: np.ndarray) -> np.ndarray:
    out = []
    for q in p:
        if not any(abs(abs(float(np.dot(q, r))) - 1.0) < 1e-9 for r in out):
            out.append(q)
    return np.array(out)


def spring_table(n_springs: int):
    """Spring directions and weights.

    Returns ``dirs`` float64 [N_s, 6] (Voigt order xx, yy, zz, xy, yz, zx with
    engineering shear: the engineering shear strain of spring k is
    ``dirs[k] @ eps``) and ``weights`` float64 [N_s] (all 5 / N_s).

    * N_s = 150: the 15 two-fold axes of the icosahedron as plane normals a,
      each with 10 slip directions b at 18 degree steps.
    * N_s = 12: the 6 five-fold axes, each with 2 slip directions 90 degrees
      apart.
    The in-plane basis is t = normalize(a x e_x) (a x e_y if |a_x| > 0.9),
    u = a x t; b_m = cos(m*step) t + sin(m*step) u.
    """
    v = _icosahedron_vertices()
    if n_springs == 150:
        d = np.linalg.norm(v[:, None] - v[None], axis=2)
        mind = np.min(d[d > 1e-9])
        mids = np.array([v[i] + v[j] for i in range(12) for j in range(i + 1, 12)
                         if abs(d[i, j] - mind) < 1e-9])
        axes = _merge_antipodes(mids / np.linalg.norm(mids, axis=1)[:, None])
        nslip, step = 10, math.pi / 10
    elif n_springs == 12:
        axes = _merge_antipodes(v)
        nslip, step = 2, math.pi / 2
    else:
        raise ValueError("spring table defined for N_s in {12, 150}")
    rows = []
    ex, ey = np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    for a in axes:
        t = np.cross(a, ey if abs(a[0]) > 0.9 else ex)
        t /= np.linalg.norm(t)
        u = np.cross(a, t)
        for mm in range(nslip):
            b = math.cos(mm * step) * t + math.sin(mm * step) * u
            rows.append([2 * a[0] * b[0], 2 * a[1] * b[1], 2 * a[2] * b[2],
                         a[0] * b[1] + a[1] * b[0], a[1] * b[2] + a[2] * b[1],
                         a[2] * b[0] + a[0] * b[2]])
    dirs = np.ascontiguousarray(np.array(rows, float))
    weights = np.full(dirs.shape[0], 5.0 / dirs.shape[0])
    return dirs, weights


# --------------------------------------------------------------------------
# Input waves
# --------------------------------------------------------------------------

def band_limited_wave(seed: int, n_steps: int, dt: float, f_lo: float = 0.1,
                      f_hi: float = 10.0, peak: float = 2.0, ramp: int = 50) -> np.ndarray:
    """Seeded band-limited Gaussian acceleration history of length n_steps."""
    L = max(65536, 4 * n_steps)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(L)
    F = np.fft.rfft(w)
    f = np.fft.rfftfreq(L, d=dt)
    F[(f < f_lo) | (f > f_hi)] = 0.0
    x = np.fft.irfft(F, n=L)[:n_steps].copy()
    r = min(ramp, n_steps)
    if r > 0:
        x[:r] *= 0.5 * (1.0 - np.cos(np.pi * np.arange(r) / r))
    mx = np.max(np.abs(x))
    return x * (peak / mx) if mx > 0 else x


def member_waves(config: int, members, n_steps: int, dt: float, peak_xy: float = 2.0,
                 peak_z: float = 1.0) -> np.ndarray:
    """[len(members), n_steps, 3] incident accelerations, seed 1e6*c + 1e3*m + k."""
    out = np.zeros((len(members), n_steps, 3))
    for i, m in enumerate(members):
        for k in range(3):
            out[i, :, k] = band_limited_wave(1_000_000 * config + 1000 * m + k, n_steps, dt,
                                             peak=peak_xy if k < 2 else peak_z)
    return out


# --------------------------------------------------------------------------
# Problem assembly (plain data)
# --------------------------------------------------------------------------

@dataclass
class Problem:
    """Plain problem data matching the C-ABI problem struct."""

    n_members: int
    n_layers: int
    rho: np.ndarray        # [n_members, n_layers]
    vs: np.ndarray
    nu: np.ndarray
    gamma_ref: np.ndarray
    h_max: np.ndarray      # [n_layers]
    nonlinear: np.ndarray  # int32 [n_layers]
    dirs: np.ndarray       # [N_s, 6]
    weights: np.ndarray    # [N_s]
    dt: float
    n_steps: int
    input_acc: np.ndarray  # [n_members, n_steps, 3]
    damping_mode: int = DAMPING_LAW
    h0: float = 0.0
    f_lo: float = 0.1
    f_hi: float = 10.0
    cg_tol: float = 1e-8
    cg_maxit: int = 5000
    precision: int = PRECISION_FP64
    inner_tol: float = 0.1
    inner_maxit: int = 50
    inner_dtype: int = 0   # 0: bfloat16 D for the inner operator, 1: FP32
    masing_depth: int = 1  # reversal points the law remembers (1: three rules; K > 1: inner loops close)

    @property
    def n_springs(self) -> int:
        return int(self.dirs.shape[0])


CFG0_LAYERS = dict(vs=(150.0, 400.0), rho=(1700.0, 1900.0))


def make_problem(n_members: int, vs_layers, rho_layers, nu: float = 0.45, gamma_ref=1e-3,
                 h_max: float = 0.2, n_springs: int = 150, dt: float = 1e-3, n_steps: int = 200,
                 input_acc=None, **kw) -> Problem:
    nl = len(vs_layers)
    vs = np.tile(np.asarray(vs_layers, float), (n_members, 1))
    rho = np.tile(np.asarray(rho_layers, float), (n_members, 1))
    g = np.asarray(gamma_ref, float)
    if g.ndim == 0:
        g = np.full((n_members, nl), float(g))
    elif g.ndim == 1:
        g = np.tile(g[:, None], (1, nl))
    dirs, w = spring_table(n_springs)
    if input_acc is None:
        input_acc = np.zeros((n_members, n_steps, 3))
    return Problem(n_members=n_members, n_layers=nl, rho=rho, vs=vs,
                   nu=np.full((n_members, nl), nu), gamma_ref=g,
                   h_max=np.full(nl, h_max), nonlinear=np.ones(nl, np.int32),
                   dirs=dirs, weights=w, dt=dt, n_steps=n_steps,
                   input_acc=np.ascontiguousarray(input_acc, float), **kw)


def ensemble_members(seed_base: int, n_members: int, vs0, sigma: float = 0.2,
                     gref_lo: float = 5e-4, gref_hi: float = 2e-3):
    """Per-member layer Vs (lognormal about ``vs0``) and gamma_ref (uniform)."""
    vs = np.zeros((n_members, len(vs0)))
    gr = np.zeros(n_members)
    for m in range(n_members):
        rng = np.random.default_rng(seed_base + m)
        xi = rng.standard_normal(len(vs0))
        vs[m] = np.asarray(vs0) * np.exp(sigma * xi)
        gr[m] = rng.uniform(gref_lo, gref_hi)
    return vs, gr


def config(c: int, n_steps: int | None = None, n_members: int | None = None,
           mesh_dims=None, recv_stride: int | None = None, **kw):
    """(mesh, problem) for workload ``c`` in 0..3 (4 is a request stream).

    Sizes can be reduced through the keyword overrides for tests; the
    defaults are the full workloads:
      0: 16x16x8 cubes, 2 layers, N_s 150, 1 member, 200 steps, FP64.
      1: 128x128x32 cubes, 3 perturbed layers, N_s 150, 1 member, 2000 steps.
      2: 64x64x32 cubes, config-0 layers, N_s 12, 64 members, 1500 steps, mixed.
      3: as 2 with 512 members, 100 steps.
    """
    dt = 1e-3
    if c == 0:
        dims = mesh_dims or (16, 16, 8)
        mesh = box_mesh(*dims, 1.0, two_layer(4.0), recv_stride or 1)
        ns = n_steps or 200
        nm = n_members or 1
        acc = member_waves(0, range(nm), ns, dt)
        prob = make_problem(nm, CFG0_LAYERS["vs"], CFG0_LAYERS["rho"], n_springs=kw.pop("n_springs", 150),
                            n_steps=ns, input_acc=acc, **kw)
        return mesh, prob
    if c == 1:
        dims = mesh_dims or (128, 128, 32)
        mesh = perturbed_three_layer_mesh(*dims, seed=1_000_001, recv_stride=recv_stride or 4)
        ns = n_steps or 2000
        acc = member_waves(1, range(1), ns, dt)
        prob = make_problem(1, (150.0, 250.0, 400.0), (1700.0, 1800.0, 1900.0),
                            n_springs=kw.pop("n_springs", 150), n_steps=ns, input_acc=acc, **kw)
        return mesh, prob
    if c in (2, 3):
        dims = mesh_dims or (64, 64, 32)
        mesh = box_mesh(*dims, 1.0, two_layer(4.0), recv_stride or 4)
        nm = n_members or (64 if c == 2 else 512)
        ns = n_steps or (1500 if c == 2 else 100)
        vs, gr = ensemble_members(2000 if c == 2 else 3000, nm, CFG0_LAYERS["vs"])
        acc = member_waves(c, range(nm), ns, dt)
        kw.setdefault("precision", PRECISION_MIXED)
        prob = make_problem(nm, CFG0_LAYERS["vs"], CFG0_LAYERS["rho"], gamma_ref=gr,
                            n_springs=kw.pop("n_springs", 12), n_steps=ns, input_acc=acc, **kw)
        prob.vs = np.ascontiguousarray(vs)
        return mesh, prob
    raise ValueError(c)


def serving_mesh(n: int, recv_stride: int = 4) -> Mesh:
    """Request mesh of the serving stream: n x n x 16 one-metre cubes with the
    config-0 layers."""
    return box_mesh(n, n, 16, 1.0, two_layer(4.0), recv_stride)


def serving_problem(req: dict, precision: int = PRECISION_MIXED, **kw) -> Problem:
    """Problem of one serving request: one member, its own layer Vs and wave
    (seeded by the request index), gamma_ref 1e-3, 12 springs."""
    acc = member_waves(4, [req["wave_seed_member"]], req["steps"], 1e-3)
    prob = make_problem(1, CFG0_LAYERS["vs"], CFG0_LAYERS["rho"], n_springs=12, n_steps=req["steps"],
                        input_acc=acc, precision=precision, **kw)
    prob.vs = np.ascontiguousarray(np.asarray(req["vs"], float)[None, :])
    return prob


def serving_requests(rate: float = 4.0, window_s: float = 60.0, seed: int = 4000,
                     sizes=(32, 48, 64), steps_range=(500, 2000)):
    """Poisson request stream: list of dicts (t_arrival, n, steps, vs, seed)."""
    rng = np.random.default_rng(seed)
    t, out, i = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window_s:
            break
        n = int(rng.choice(sizes))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        xi = rng.standard_normal(2)
        vs = np.asarray(CFG0_LAYERS["vs"]) * np.exp(0.2 * xi)
        out.append(dict(t=t, n=n, steps=steps, vs=vs, wave_seed_member=i))
        i += 1
    return out
