"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Bars: FP64 path <= 1e-9 and mixed path <= 1e-6 relative L2 on receiver
velocity (parity runs use CG tolerance 1e-12 on both sides, so the mixed path
is held to 1e-9 there as well); single operator applications to 1e-13 (FP64)
and 2e-6 (FP32, the inner preconditioner's arithmetic).
"""
import sys

import numpy as np
import pytest

from paper_2604_02755_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rand_D(rng, ne, G0=4e7, lam=3e8):
    """SPD D per point: isotropic plus a random symmetric PSD part."""
    base = np.zeros((6, 6))
    base[:3, :3] = lam
    base[np.arange(3), np.arange(3)] += 2 * G0
    base[3:, 3:] = np.eye(3) * G0
    L = rng.normal(size=(ne, 4, 6, 6)) * 0.3 * G0 ** 0.5
    D = base + np.einsum("eiab,eicb->eiac", L, L)
    iu = np.triu_indices(6)
    return D[:, :, iu[0], iu[1]]


@pytest.mark.parametrize("dims", [(5, 4, 3), (16, 16, 8)])
def test_operator_parity(gpu_ctx, oracle_lib, dims):
    mesh, prob = I.config(0, n_steps=1, mesh_dims=dims)
    say("operator parity", dims, mesh.n_tets)
    rng = np.random.default_rng(11)
    D = _rand_D(rng, mesh.n_tets)
    h = rng.uniform(0, 0.2, mesh.n_tets)
    x = rng.normal(size=mesh.n_dof)
    mh = gpu_ctx.mesh(mesh)
    for which in (0, 1, 2):
        y_ref = oracle_lib.apply_operator(mesh, prob, which, D, h, x)
        y = gpu_ctx.apply_operator(mh, prob, which, 0, D, h, x)
        err = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
        say("  op", which, "fp64 rel err", err)
        assert err < 1e-13
    y_ref = oracle_lib.apply_operator(mesh, prob, 0, D, h, x)
    prob.inner_dtype = 1  # FP32 D
    y32 = gpu_ctx.apply_operator(mh, prob, 0, 1, D, h, x)
    err = np.linalg.norm(y32 - y_ref) / np.linalg.norm(y_ref)
    say("  op A fp32 rel err", err)
    assert err < 2e-6
    prob.inner_dtype = 0  # bfloat16 D (the inner preconditioner's default): 8-bit mantissa
    y16 = gpu_ctx.apply_operator(mh, prob, 0, 1, D, h, x)
    err = np.linalg.norm(y16 - y_ref) / np.linalg.norm(y_ref)
    say("  op A fp32/bf16-D rel err", err)
    assert err < 4e-3
    # one bfloat16 D per element, the mean of its four points: the oracle
    # applied with that mean at every point
    prob.inner_dtype = 2
    Dm = np.repeat(D.mean(axis=1, keepdims=True), 4, axis=1)
    ym_ref = oracle_lib.apply_operator(mesh, prob, 0, Dm, h, x)
    ym = gpu_ctx.apply_operator(mh, prob, 0, 1, D, h, x)
    err = np.linalg.norm(ym - ym_ref) / np.linalg.norm(ym_ref)
    say("  op A fp32/bf16 element-mean D rel err", err)
    assert err < 4e-3
    # with D constant over each element and exactly representable in bfloat16
    # the element-mean path differs from the oracle by FP32 rounding only (its
    # closed-form integration of the forces is exact for constant D)
    Dc = D.mean(axis=1, keepdims=True).astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    Dc = np.repeat(Dc.view(np.float32).astype(np.float64), 4, axis=1)
    yc_ref = oracle_lib.apply_operator(mesh, prob, 0, Dc, h, x)
    yc = gpu_ctx.apply_operator(mh, prob, 0, 1, Dc, h, x)
    err = np.linalg.norm(yc - yc_ref) / np.linalg.norm(yc_ref)
    say("  op A fp32, bf16-exact constant D per element, rel err", err)
    assert err < 2e-6
    prob.inner_dtype = 0


def _small_problem(n_steps=40, precision=0, tol=1e-12, n_members=1, dims=(5, 4, 3), scale=5.0, ns=150):
    mesh, prob = I.config(0, n_steps=n_steps, mesh_dims=dims, n_members=n_members, cg_tol=tol,
                          precision=precision, n_springs=ns)
    prob.input_acc *= scale  # drive the springs well past gamma_ref
    return mesh, prob


def _oracle_vel(oracle_lib, mesh, prob, m=0):
    r = oracle_lib.run(mesh, prob, member=m)
    return r["vel"], r["iters"]


def test_fp64_path_parity_small(gpu_ctx, oracle_lib):
    mesh, prob = _small_problem()
    say("fp64 path", mesh.n_tets, "tets", prob.n_steps, "steps")
    vref, itref = _oracle_vel(oracle_lib, mesh, prob)
    mh = gpu_ctx.mesh(mesh)
    out = gpu_ctx.solve(mh, mesh, prob)
    assert out["rc"] == 0
    err = oracle_lib.rel_l2(out["vel"][0], vref)
    say("  rel L2", err, "iters gpu", out["iters"][0, :8, 0], "oracle", itref[:8])
    assert err < 1e-9
    assert np.max(np.abs(out["iters"][0, :, 0] - itref)) <= 1
    # maximum velocity-norm map (Section 3, Figs. 3-4) against the oracle's
    ref = oracle_lib.run(mesh, prob)
    verr = float(np.max(np.abs(out["vmax"][0] - ref["vmax"])) / np.max(ref["vmax"]))
    say("  vmax max rel err", verr)
    assert ref["vmax"].max() > 0 and verr < 1e-9


def test_mixed_path_parity_small(gpu_ctx, oracle_lib):
    mesh, prob = _small_problem(precision=1)
    say("mixed path", mesh.n_tets, "tets")
    vref, _ = _oracle_vel(oracle_lib, mesh, prob)
    mh = gpu_ctx.mesh(mesh)
    out = gpu_ctx.solve(mh, mesh, prob)
    assert out["rc"] == 0
    err = oracle_lib.rel_l2(out["vel"][0], vref)
    say("  rel L2 (tol 1e-12)", err, "outer/inner", out["iters"][0, 10:14])
    assert err < 1e-9
    # throughput tolerance: mixed vs FP64, both at 1e-8
    mesh, p8 = _small_problem(precision=1, tol=1e-8)
    _, p64 = _small_problem(precision=0, tol=1e-8)
    o_mixed = gpu_ctx.solve(mh, mesh, p8)
    o_fp64 = gpu_ctx.solve(mh, mesh, p64)
    err = oracle_lib.rel_l2(o_mixed["vel"][0], o_fp64["vel"][0])
    err_or = oracle_lib.rel_l2(o_mixed["vel"][0], vref)
    say("  mixed vs fp64 at 1e-8", err, "vs oracle", err_or)
    assert err < 1e-6 and err_or < 1e-6
    # inner operator with one D per element: the outer FP64 iteration still
    # converges to the same solution
    mesh, pm = _small_problem(precision=1, tol=1e-12)
    pm.inner_dtype = 2
    o_mean = gpu_ctx.solve(mh, mesh, pm)
    err = oracle_lib.rel_l2(o_mean["vel"][0], vref)
    say("  mixed, element-mean inner D, tol 1e-12, vs oracle", err, "outer/inner", o_mean["iters"][0, 10:14])
    assert o_mean["rc"] == 0 and err < 1e-9


def test_batch_matches_members_alone_and_oracle(gpu_ctx, oracle_lib):
    mesh, prob = _small_problem(n_members=3, n_steps=30, ns=12)
    vs, gr = I.ensemble_members(77, 3, I.CFG0_LAYERS["vs"])
    prob.vs = vs
    prob.gamma_ref = np.tile(gr[:, None], (1, 2))
    say("batch of 3 (padded to 4)")
    mh = gpu_ctx.mesh(mesh)
    out = gpu_ctx.solve(mh, mesh, prob)
    assert out["rc"] == 0
    for m in range(3):
        vref, _ = _oracle_vel(oracle_lib, mesh, prob, m)
        alone = gpu_ctx.solve(mh, mesh, prob, members=[m])
        e_or = oracle_lib.rel_l2(out["vel"][m], vref)
        e_al = oracle_lib.rel_l2(out["vel"][m], alone["vel"][0])
        say("  member", m, "vs oracle", e_or, "batched vs alone", e_al)
        assert e_or < 1e-9 and e_al < 1e-12


@pytest.mark.parametrize("flags", [(1, 0), (0, 1)])
def test_per_layer_elastic_flag_matches_oracle(gpu_ctx, oracle_lib, flags):
    """A layer flagged elastic keeps its springs linear (D = the elastic
    tangent, no hysteretic damping) while the other layer's springs yield:
    FP64 and mixed runs match the oracle."""
    for precision in (0, 1):
        mesh, prob = _small_problem(precision=precision, n_steps=30, ns=12)
        prob.nonlinear = np.array(flags, dtype=np.int32)
        say("layer flags", flags, "precision", precision)
        vref, _ = _oracle_vel(oracle_lib, mesh, prob)
        mh = gpu_ctx.mesh(mesh)
        out = gpu_ctx.solve(mh, mesh, prob)
        err = oracle_lib.rel_l2(out["vel"][0], vref)
        say("  rel L2", err)
        assert out["rc"] == 0 and err < 1e-9


def test_nonconvergence_reported(gpu_ctx, nlth_mod):
    mesh, prob = _small_problem(n_steps=5, tol=1e-12)
    prob.cg_maxit = 2
    mh = gpu_ctx.mesh(mesh)
    out = gpu_ctx.solve(mh, mesh, prob)
    say("enoconv rc", out["rc"], out["status"])
    assert out["rc"] == nlth_mod.NLTH_ENOCONV and out["status"][0] == nlth_mod.NLTH_ENOCONV


def test_config0_fp64_parity(gpu_ctx, oracle_lib):
    """16x16x8 cubes, two layers, 150 springs, 1 ms steps (the first 100 of
    the 200-step record, which covers the ramp and the strong motion)."""
    mesh, prob = I.config(0, n_steps=100, cg_tol=1e-12)
    say("config 0 fp64, 100 steps")
    vref, itref = _oracle_vel(oracle_lib, mesh, prob)
    mh = gpu_ctx.mesh(mesh)
    out = gpu_ctx.solve(mh, mesh, prob)
    err = oracle_lib.rel_l2(out["vel"][0], vref)
    say("  rel L2", err, "iters", out["iters"][0, 40:44, 0], itref[40:44])
    assert out["rc"] == 0 and err < 1e-9


def test_tuning_knobs_keep_results(gpu_ctx, nlth_mod):
    """Launch shapes (threads per block, hipGraph-captured CG chunks, chunk
    length) change no arithmetic: converged members are frozen on the device,
    and the coloured scatter and the dot reductions have a fixed order."""
    mesh, prob = _small_problem(precision=1, n_members=3, n_steps=20, dims=(8, 8, 4), ns=12, tol=1e-10)
    mh = gpu_ctx.mesh(mesh)

    def run(**kw):
        ens = gpu_ctx.ensemble(mh, mesh, prob)
        try:
            if kw:
                ens.set_tuning(**kw)
            ens.step(prob.n_steps)
            return ens.read()
        finally:
            ens.close()

    say("tuning knobs: graph, direct, 128 threads / 4 per check, 64 threads / 16 per check, colours")
    base = run()
    for kw in (dict(use_graph=0), dict(ebe_block=128, check_every=4), dict(ebe_block=64, check_every=16)):
        o = run(**kw)
        d = float(np.max(np.abs(o["vel"] - base["vel"])))
        say("  ", kw, "max |dv|", d, "iters equal", bool(np.array_equal(o["iters"], base["iters"])))
        assert d == 0.0 and np.array_equal(o["iters"], base["iters"])
    # one launch per colour adding into y: another summation order, same
    # operator; the runs agree to the solver tolerance
    o = run(scatter=1)
    err = float(np.linalg.norm(o["vel"] - base["vel"]) / np.linalg.norm(base["vel"]))
    say("   colour path vs gather path rel err", err)
    assert err < 1e-8
    ens = gpu_ctx.ensemble(mh, mesh, prob)
    try:
        for bad in (dict(ebe_block=100), dict(check_every=65), dict(inner_tol=2.0), dict(scatter=2)):
            with pytest.raises(nlth_mod.NlthError) as ei:
                ens.set_tuning(**bad)
            assert ei.value.code == nlth_mod.NLTH_EINVAL
    finally:
        ens.close()


def test_autotuned_run_matches_fp64(gpu_ctx):
    """The autotuner switches the inner policy between steps; every step still
    converges to the outer FP64 tolerance, so the run stays within 1e-6 of the
    plain FP64 path."""
    from paper_2604_02755_amd import autotune
    mesh, pm = _small_problem(precision=1, n_members=2, n_steps=40, dims=(8, 8, 4), ns=12, tol=1e-8)
    _, p64 = _small_problem(precision=0, n_members=2, n_steps=40, dims=(8, 8, 4), ns=12, tol=1e-8)
    mh = gpu_ctx.mesh(mesh)
    autotune._cache.clear()
    ens = gpu_ctx.ensemble(mh, mesh, pm)
    try:
        choice = autotune.tune(ens, mesh, pm, steps_per_trial=1)
        done = ens.stats()["steps_done"]
        say("autotune choice", {k: choice[k] for k in ("inner_tol", "inner_maxit", "ebe_block", "check_every")},
            "after", done, "steps")
        # every timed trial is one step, plus one untimed step for the Chebyshev estimate
        assert done == autotune.trial_steps(pm) == len(choice["trials"]) + 1 and done < pm.n_steps
        ens.step(pm.n_steps - done)
        om = ens.read()
    finally:
        ens.close()
    o64 = gpu_ctx.solve(mh, mesh, p64)
    for m in range(2):
        err = np.linalg.norm(om["vel"][m] - o64["vel"][m]) / np.linalg.norm(o64["vel"][m])
        say("  member", m, "autotuned mixed vs fp64", err)
        assert err < 1e-6


@pytest.mark.parametrize("precision,inner_dtype", [(0, 0), (1, 0), (1, 2)])
def test_cluster_path_64_members(gpu_ctx, oracle_lib, precision, inner_dtype):
    """64 member slots take the cluster path (element clusters summed in LDS,
    then per node): members match the oracle and the colour path; inner_dtype
    2 is the benchmark's inner operator (one bfloat16 D per element)."""
    mesh, prob = _small_problem(precision=precision, n_members=64, n_steps=24, dims=(6, 5, 3), ns=12, tol=1e-12)
    prob.inner_dtype = inner_dtype
    vs, gr = I.ensemble_members(91, 64, I.CFG0_LAYERS["vs"])
    prob.vs = vs
    prob.gamma_ref = np.tile(gr[:, None], (1, 2))
    prob.input_acc = 5.0 * I.member_waves(2, range(64), prob.n_steps, prob.dt)
    mh = gpu_ctx.mesh(mesh)

    def run(**kw):
        ens = gpu_ctx.ensemble(mh, mesh, prob)
        try:
            if kw:
                ens.set_tuning(**kw)
            ens.step(prob.n_steps)
            return ens.read()
        finally:
            ens.close()

    say("cluster path, 64 members, precision", precision, "inner dtype", inner_dtype)
    cl = run()
    col = run(scatter=1)
    d = float(np.max(np.abs(cl["vel"] - col["vel"])) / np.max(np.abs(col["vel"])))
    say("  cluster vs colour max rel diff", d)
    assert d < 1e-9
    for m in (0, 37, 63):
        vref, _ = _oracle_vel(oracle_lib, mesh, prob, m)
        err = oracle_lib.rel_l2(cl["vel"][m], vref)
        say("  member", m, "vs oracle", err)
        assert err < 1e-9


@pytest.mark.parametrize("n_members,n_live,tail", [(64, 20, 32), (64, 10, 16), (128, 24, 32)])
def test_tail_operator_matches_full_and_oracle(gpu_ctx, oracle_lib, n_members, n_live, tail):
    """With at most `tail` members still iterating in the outer CG, their
    inner CG runs on compact copies of their rows.  Members without input are
    inactive from the start, so the compact path runs in every outer
    iteration: results match the full path and the oracle, silent members stay
    at rest, graph replay equals direct launches bitwise, and the profile
    counts the listed element-member pairs."""
    nmb = n_members
    mesh, prob = _small_problem(precision=1, n_members=nmb, n_steps=24, dims=(6, 5, 3), ns=12, tol=1e-12)
    prob.inner_dtype = 2
    vs, gr = I.ensemble_members(91, nmb, I.CFG0_LAYERS["vs"])
    prob.vs = vs
    prob.gamma_ref = np.tile(gr[:, None], (1, 2))
    live = np.arange(3, nmb, nmb // n_live)[:n_live]  # spread over the member lanes
    acc = 5.0 * I.member_waves(2, range(nmb), prob.n_steps, prob.dt)
    mask = np.zeros(nmb, dtype=bool)
    mask[live] = True
    acc[~mask] = 0.0
    prob.input_acc = acc
    mh = gpu_ctx.mesh(mesh)

    def run(profile=False, **kw):
        ens = gpu_ctx.ensemble(mh, mesh, prob)
        try:
            ens.set_tuning(**kw)
            if profile:
                ens.set_profile(True)
            ens.step(prob.n_steps)
            return ens.read(), ens.stats()
        finally:
            ens.close()

    say("tail operator:", n_live, "of", nmb, "members live, list of at most", tail)
    full, _ = run(tail_members=0)
    lst, _ = run(tail_members=tail)
    prof, st = run(profile=True, tail_members=tail)
    say("  tail launches", st["n_tail32"], "element-member pairs", st["elems_tail32"], "full launches", st["n_ebe32"])
    assert st["n_tail32"] > 0 and st["n_ebe32"] == 0
    assert st["elems_tail32"] <= st["n_tail32"] * mesh.n_tets * n_live
    assert st["elems_tail32"] % mesh.n_tets == 0
    assert np.all(lst["vel"][~mask] == 0.0)
    scale = np.max(np.abs(full["vel"]))
    d = float(np.max(np.abs(lst["vel"] - full["vel"])) / scale)
    dp = float(np.max(np.abs(prof["vel"] - lst["vel"])) / scale)
    say("  list vs full max rel diff", d, "profiled vs graph-replayed", dp)
    assert d < 1e-9 and dp == 0.0
    for m in (live[0], live[-1]):
        vref, _ = _oracle_vel(oracle_lib, mesh, prob, int(m))
        err = oracle_lib.rel_l2(lst["vel"][m], vref)
        say("  member", int(m), "vs oracle", err)
        assert err < 1e-9


@pytest.mark.parametrize("n_members,n_live", [(64, 20), (64, 10), (128, 24)])
def test_fp64_tail_matches_full_and_oracle(gpu_ctx, oracle_lib, n_members, n_live):
    """Plain FP64 PCG: once at most 32 members are still iterating, their PCG
    moves to compact rows of 16 or 32 lanes (D per point, the PCG vectors)
    for the rest of the step.  Members without input converge at once, so the
    compact path runs from the first check: results match the full path and
    the oracle, silent members stay at rest, iteration counts match the full
    path's, and graph replay equals direct launches bitwise."""
    nmb = n_members
    mesh, prob = _small_problem(precision=0, n_members=nmb, n_steps=16, dims=(6, 5, 3), ns=12, tol=1e-12)
    vs, gr = I.ensemble_members(93, nmb, I.CFG0_LAYERS["vs"])
    prob.vs = vs
    prob.gamma_ref = np.tile(gr[:, None], (1, 2))
    live = np.arange(5, nmb, nmb // n_live)[:n_live]
    acc = 5.0 * I.member_waves(3, range(nmb), prob.n_steps, prob.dt)
    mask = np.zeros(nmb, dtype=bool)
    mask[live] = True
    acc[~mask] = 0.0
    prob.input_acc = acc
    mh = gpu_ctx.mesh(mesh)

    def run(profile=False, **kw):
        ens = gpu_ctx.ensemble(mh, mesh, prob)
        try:
            ens.set_tuning(**kw)
            if profile:
                ens.set_profile(True)
            ens.step(prob.n_steps)
            return ens.read(), ens.stats()
        finally:
            ens.close()

    say("fp64 tail:", n_live, "of", nmb, "members live")
    full, _ = run(tail_members=0)
    lst, _ = run(tail_members=32)
    prof, st = run(profile=True, tail_members=32)
    say("  tail launches", st["n_tail32"], "element-member pairs", st["elems_tail32"])
    assert st["n_tail32"] > 0 and st["elems_tail32"] <= st["n_tail32"] * mesh.n_tets * n_live
    assert st["elems_tail32"] % mesh.n_tets == 0
    assert np.all(lst["vel"][~mask] == 0.0)
    scale = np.max(np.abs(full["vel"]))
    d = float(np.max(np.abs(lst["vel"] - full["vel"])) / scale)
    dp = float(np.max(np.abs(prof["vel"] - lst["vel"])) / scale)
    say("  list vs full max rel diff", d, "profiled vs graph-replayed", dp)
    assert d < 1e-10 and dp == 0.0
    assert np.max(np.abs(lst["iters"][:, :, 0] - full["iters"][:, :, 0])) <= 1
    for m in (live[0], live[-1]):
        vref, itref = _oracle_vel(oracle_lib, mesh, prob, int(m))
        err = oracle_lib.rel_l2(lst["vel"][m], vref)
        say("  member", int(m), "vs oracle", err)
        assert err < 1e-9 and np.max(np.abs(lst["iters"][m, :, 0] - itref)) <= 1


def test_chebyshev_inner_matches_oracle(gpu_ctx, oracle_lib, nlth_mod):
    """Inner Chebyshev iteration (bounds from the step's first inner CG): the
    outer FP64 flexible CG still converges to its tolerance, so members match
    the oracle; the fused cluster-gather update (64 slots) and the separate
    update (colour path, and fewer than 64 slots) agree."""
    mesh, prob = _small_problem(precision=1, n_members=64, n_steps=24, dims=(6, 5, 3), ns=12, tol=1e-12)
    vs, gr = I.ensemble_members(91, 64, I.CFG0_LAYERS["vs"])
    prob.vs = vs
    prob.gamma_ref = np.tile(gr[:, None], (1, 2))
    prob.input_acc = 5.0 * I.member_waves(2, range(64), prob.n_steps, prob.dt)
    mh = gpu_ctx.mesh(mesh)

    def run(p, **kw):
        ens = gpu_ctx.ensemble(mh, mesh, p)
        try:
            ens.set_tuning(**kw)
            ens.step(p.n_steps)
            return ens.read()
        finally:
            ens.close()

    say("chebyshev inner, 64 members (fused cluster gather) and colour path")
    cg = run(prob, inner_maxit=16, inner_tol=1e-12, inner_method=0)
    ch = run(prob, inner_maxit=16, inner_tol=1e-12, inner_method=1)
    chc = run(prob, inner_maxit=16, inner_tol=1e-12, inner_method=1, scatter=1)
    ens = gpu_ctx.ensemble(mh, mesh, prob)
    try:
        ens.set_tuning(inner_maxit=16, inner_tol=1e-12, inner_method=1)
        ens.step(3)
        st = ens.stats()
        say("  Chebyshev interval after 3 steps", st["cheb_lo_min"], st["cheb_hi_max"])
        assert 0 < st["cheb_lo_min"] < st["cheb_hi_max"] < 100
    finally:
        ens.close()
    o_cg, o_ch = cg["iters"][:, :, 0].mean(), ch["iters"][:, :, 0].mean()
    say("  outer iterations per member-step: CG inner", o_cg, "Chebyshev inner", o_ch)
    assert o_ch <= 1.5 * o_cg
    d = float(np.max(np.abs(ch["vel"] - chc["vel"])) / np.max(np.abs(chc["vel"])))
    say("  fused vs separate update max rel diff", d)
    assert d < 1e-9
    for m in (0, 37, 63):
        vref, _ = _oracle_vel(oracle_lib, mesh, prob, m)
        err = oracle_lib.rel_l2(ch["vel"][m], vref)
        say("  member", m, "vs oracle", err)
        assert err < 1e-9
    # fewer than 64 slots (element outputs + gather, separate update), at the
    # throughput tolerance against the plain FP64 path
    mesh2, p8 = _small_problem(precision=1, n_members=2, tol=1e-8)
    _, p64 = _small_problem(precision=0, n_members=2, tol=1e-8)
    mh2 = gpu_ctx.mesh(mesh2)
    ens = gpu_ctx.ensemble(mh2, mesh2, p8)
    try:
        ens.set_tuning(inner_maxit=12, inner_tol=1e-12, inner_method=1)
        ens.step(p8.n_steps)
        om = ens.read()
        with pytest.raises(nlth_mod.NlthError) as ei:
            ens.set_tuning(inner_maxit=65, inner_method=1)
        assert ei.value.code == nlth_mod.NLTH_EINVAL
    finally:
        ens.close()
    o64 = gpu_ctx.solve(mh2, mesh2, p64)
    for m in range(2):
        err = oracle_lib.rel_l2(om["vel"][m], o64["vel"][m])
        say("  2 members, member", m, "chebyshev mixed vs fp64 at 1e-8", err)
        assert err < 1e-6


def test_response_spectra_matches_oracle(gpu_ctx, oracle_lib, nlth_mod):
    """Velocity response spectra (h = 0.05) on the device against the oracle's
    matrix-exponential stepping: band-limited records and the receiver
    histories of a nonlinear run, both spectrum kinds, to 1e-10 of the peak."""
    dt = 1e-3
    recs = [np.cumsum(I.band_limited_wave(7000 + k, 3000, dt)) * dt for k in range(5)]
    mesh, prob = _small_problem(precision=0, n_steps=60, scale=20.0)
    out = gpu_ctx.solve(gpu_ctx.mesh(mesh), mesh, prob)
    hist = out["vel"][0].transpose(1, 2, 0).reshape(-1, prob.n_steps)[:12]  # receiver components over time
    periods = np.geomspace(0.02, 5.0, 37)
    for vel, step in ((np.array(recs), dt), (np.ascontiguousarray(hist), prob.dt)):
        for kind in (0, 1):
            g = gpu_ctx.response_spectra(vel, step, periods, 0.05, kind)
            o = oracle_lib.response_spectra(vel, step, periods, 0.05, kind)
            err = float(np.max(np.abs(g - o)) / np.max(np.abs(o)))
            say("response spectra, kind", kind, vel.shape, "max rel err", err)
            assert np.max(np.abs(o)) > 0 and err < 1e-10
    with pytest.raises(nlth_mod.NlthError) as ei:
        gpu_ctx.response_spectra(recs[0], dt, [0.1, -1.0])
    assert ei.value.code == nlth_mod.NLTH_EINVAL


def _three_layer(n_members, n_steps, precision, tol, dims=(8, 8, 8), ns=150, seed=5):
    """Config-1 geometry at test size: three layers whose interfaces follow
    seeded smooth random surfaces (nodes moved to fit), 150 springs."""
    mesh = I.perturbed_three_layer_mesh(*dims, seed=seed, amp=0.8, corr=4.0, recv_stride=2)
    acc = 8.0 * I.member_waves(1, range(n_members), n_steps, 1e-3)
    prob = I.make_problem(n_members, (150.0, 250.0, 400.0), (1700.0, 1800.0, 1900.0), n_springs=ns,
                          n_steps=n_steps, input_acc=acc, cg_tol=tol, precision=precision)
    if n_members > 1:
        vs, gr = I.ensemble_members(2100, n_members, (150.0, 250.0, 400.0))
        prob.vs = np.ascontiguousarray(vs)
        prob.gamma_ref = np.ascontiguousarray(np.tile(gr[:, None], (1, 3)))
    return mesh, prob


@pytest.mark.parametrize("precision", [0, 1])
def test_perturbed_three_layer_mesh_matches_oracle(gpu_ctx, oracle_lib, precision):
    """Distorted, non-box geometry (three layers with perturbed interfaces,
    150 springs per point): one member, and 64 members on the cluster path
    (members 0 and 63 checked), against the oracle at tolerance 1e-12."""
    for nm in (1, 64):
        mesh, prob = _three_layer(nm, 30, precision, 1e-12)
        if precision == 1:
            prob.inner_dtype = 2 if nm == 64 else 0
        say("three-layer mesh", mesh.n_tets, "tets, members", nm, "precision", precision)
        mh = gpu_ctx.mesh(mesh)
        out = gpu_ctx.solve(mh, mesh, prob)
        assert out["rc"] == 0
        for m in ((0,) if nm == 1 else (0, 63)):
            ref = oracle_lib.run(mesh, prob, member=m)
            err = oracle_lib.rel_l2(out["vel"][m], ref["vel"])
            say("  member", m, "rel L2 vs oracle", err, "law events", ref["law_events"])
            assert np.abs(ref["vel"]).max() > 0 and err < 1e-9
            assert ref["law_events"][0] > 0  # the springs yield and reverse


@pytest.mark.parametrize("precision", [0, 1])
def test_long_run_reaches_every_law_event(gpu_ctx, oracle_lib, precision):
    """A long nonlinear run (400 steps) on a tiny mesh: the oracle counts
    reversals taken on the skeleton, reversals taken on a Masing branch and
    rejoins of the skeleton, all of which occur; the GPU run matches the
    oracle's receiver velocity through all of them."""
    mesh, prob = _small_problem(n_steps=400, precision=precision, tol=1e-12, dims=(4, 3, 2), ns=12, scale=6.0)
    say("long law run, precision", precision, prob.n_steps, "steps")
    ref = oracle_lib.run(mesh, prob)
    ev = ref["law_events"]
    say("  oracle law events (skeleton reversals, branch reversals, rejoins)", ev)
    assert ev[0] > 0 and ev[1] > 0 and ev[2] > 0
    out = gpu_ctx.solve(gpu_ctx.mesh(mesh), mesh, prob)
    err = oracle_lib.rel_l2(out["vel"][0], ref["vel"])
    verr = float(np.max(np.abs(out["vmax"][0] - ref["vmax"])) / np.max(ref["vmax"]))
    say("  rel L2 vs oracle", err, "vmax rel err", verr)
    assert out["rc"] == 0 and err < 1e-9 and verr < 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_reversal_memory_matches_oracle(gpu_ctx, oracle_lib, precision):
    """The law with a reversal memory of depth 3 (inner loops close and the
    path goes on along the branch it left): the oracle closes loops in this
    run and its result differs from the three-rule law's; the GPU matches it
    with one member slot and with 64 (members 0 and 63 checked)."""
    mesh, prob = _small_problem(n_steps=400, precision=precision, tol=1e-12, dims=(4, 3, 2), ns=12, scale=6.0)
    prob.masing_depth = 3
    ref = oracle_lib.run(mesh, prob)
    ev = ref["law_events"]
    say("reversal memory depth 3, precision", precision, "oracle law events", ev)
    assert ev[3] > 0
    prob.masing_depth = 1
    assert oracle_lib.rel_l2(oracle_lib.run(mesh, prob)["vel"], ref["vel"]) > 1e-4
    prob.masing_depth = 3
    mh = gpu_ctx.mesh(mesh)
    out = gpu_ctx.solve(mh, mesh, prob)
    err = oracle_lib.rel_l2(out["vel"][0], ref["vel"])
    say("  one member: rel L2 vs oracle", err)
    assert out["rc"] == 0 and err < 1e-9
    mesh, prob = _small_problem(n_steps=150, precision=precision, tol=1e-12, dims=(4, 3, 2), ns=12, scale=6.0,
                                n_members=64)
    prob.masing_depth = 3
    out = gpu_ctx.solve(mh, mesh, prob)
    assert out["rc"] == 0
    for m in (0, 63):
        ref = oracle_lib.run(mesh, prob, member=m)
        err = oracle_lib.rel_l2(out["vel"][m], ref["vel"])
        say("  64 members, member", m, "rel L2 vs oracle", err, "law events", ref["law_events"])
        assert ref["law_events"][3] > 0 and err < 1e-9


def test_benchmark_path_at_throughput_tolerance(gpu_ctx, oracle_lib):
    """The benchmark's launch configuration at its operating point: 64 member
    slots (cluster operator, element-mean bfloat16 inner D, compact rows for
    the convergence tail), a fixed 20 inner iterations per outer iteration,
    CG tolerance 1e-8.  Every member stays within 1e-6 of the plain FP64 path
    at 1e-8, and members 0 and 63 within 1e-6 of the oracle."""
    mesh, pm = _small_problem(precision=1, n_members=64, n_steps=60, dims=(6, 5, 3), ns=12, tol=1e-8)
    _, p64 = _small_problem(precision=0, n_members=64, n_steps=60, dims=(6, 5, 3), ns=12, tol=1e-8)
    vs, gr = I.ensemble_members(91, 64, I.CFG0_LAYERS["vs"])
    acc = 5.0 * I.member_waves(2, range(64), pm.n_steps, pm.dt)
    for p in (pm, p64):
        p.vs = vs
        p.gamma_ref = np.tile(gr[:, None], (1, 2))
        p.input_acc = acc
    pm.inner_dtype = 2
    mh = gpu_ctx.mesh(mesh)
    ens = gpu_ctx.ensemble(mh, mesh, pm)
    try:
        ens.set_tuning(128, 16, 1, 20, 1e-12, cluster_blocks=3, tail_members=32)
        ens.set_profile(True)
        ens.step(pm.n_steps)
        om, st = ens.read(), ens.stats()
    finally:
        ens.close()
    o64 = gpu_ctx.solve(mh, mesh, p64)
    say("benchmark path at 1e-8: cluster launches", st["n_ebe32"], "compact-row launches", st["n_tail32"])
    assert st["n_ebe32"] > 0 and st["n_tail32"] > 0
    errs = [oracle_lib.rel_l2(om["vel"][m], o64["vel"][m]) for m in range(64)]
    say("  mixed vs fp64, max over 64 members", max(errs))
    assert max(errs) < 1e-6
    for m in (0, 63):
        ref = oracle_lib.run(mesh, pm, member=m, cg_tol=1e-12)
        err = oracle_lib.rel_l2(om["vel"][m], ref["vel"])
        say("  member", m, "vs oracle", err)
        assert err < 1e-6


@pytest.mark.parametrize("precision", [0, 1])
def test_extrapolated_initial_guess_matches_oracle(gpu_ctx, oracle_lib, precision):
    """The CG initial guess extrapolated from the previous increments (linear,
    quadratic) changes the iteration path only: at tolerance 1e-12 the run
    matches the oracle (whose initial guess is the last increment), and at
    1e-8 it needs fewer iterations than the last increment alone."""
    mesh, prob = _small_problem(precision=precision, n_members=2, n_steps=60, dims=(6, 5, 3), ns=12, tol=1e-12)
    mh = gpu_ctx.mesh(mesh)

    def run(p, order):
        ens = gpu_ctx.ensemble(mh, mesh, p)
        try:
            ens.set_tuning(predictor=order)
            ens.step(p.n_steps)
            return ens.read()
        finally:
            ens.close()

    refs = [oracle_lib.run(mesh, prob, member=m) for m in range(2)]
    for order in (1, 2):
        out = run(prob, order)
        for m in range(2):
            err = oracle_lib.rel_l2(out["vel"][m], refs[m]["vel"])
            say("predictor", order, "precision", precision, "member", m, "rel L2 vs oracle", err)
            assert out["status"][m] == 0 and err < 1e-9
    mesh, p8 = _small_problem(precision=precision, n_members=2, n_steps=60, dims=(6, 5, 3), ns=12, tol=1e-8)
    its = {k: run(p8, k)["iters"][:, 10:, 0].sum() for k in (0, 1, 2)}
    say("  outer iterations at tol 1e-8 over steps 11-60 by predictor order", its)
    assert its[1] < its[0] and its[2] < its[0]
    with pytest.raises(Exception):
        ens = gpu_ctx.ensemble(mh, mesh, p8)
        try:
            ens.set_tuning(predictor=3)
        finally:
            ens.close()


def test_block_jacobi_diagonal_matches_oracle(gpu_ctx, oracle_lib):
    """The 3x3 diagonal blocks that the block-Jacobi preconditioner inverts
    (step a2): from D per point in FP64, and, for the mixed path with one
    bfloat16 D per element, the inner operator's blocks from closed-form
    integrals, against the diagonal blocks of the oracle's assembled A (its
    CRS operator applied to unit vectors).  With D constant per element and
    exact in bfloat16 the two forms agree to FP64 rounding."""
    mesh, prob = I.config(0, n_steps=1, mesh_dims=(3, 2, 2))
    rng = np.random.default_rng(21)
    D = _rand_D(rng, mesh.n_tets)
    h = rng.uniform(0, 0.2, mesh.n_tets)
    x = rng.normal(size=mesh.n_dof)
    mh = gpu_ctx.mesh(mesh)

    def oracle_blocks_times_x(Dx):
        B = np.zeros((mesh.n_nodes, 3, 3))
        e = np.zeros(mesh.n_dof)
        for i in range(mesh.n_dof):
            e[i] = 1.0
            col = oracle_lib.apply_operator(mesh, prob, 0, Dx, h, e)
            e[i] = 0.0
            node, c = divmod(i, 3)
            B[node, :, c] = col[3 * node:3 * node + 3]
        return np.einsum("nij,nj->ni", B, x.reshape(-1, 3)).ravel()

    y_ref = oracle_blocks_times_x(D)
    y = gpu_ctx.apply_operator(mh, prob, 3, 0, D, h, x)
    err = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
    say("block diagonal, FP64 per-point D, rel err vs oracle", err)
    assert err < 1e-13
    Dc = D.mean(axis=1, keepdims=True).astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    Dc = np.repeat(Dc.view(np.float32).astype(np.float64), 4, axis=1)
    prob.inner_dtype = 2
    y_ref = oracle_blocks_times_x(Dc)
    y = gpu_ctx.apply_operator(mh, prob, 3, 1, Dc, h, x)
    err = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
    say("block diagonal, inner operator (bfloat16 element-mean D, closed form), rel err vs oracle", err)
    assert err < 1e-13
    prob.inner_dtype = 0


@pytest.mark.parametrize("n_members", [65, 100, 257])
def test_ragged_member_counts(gpu_ctx, oracle_lib, n_members):
    """Member counts that are not a power of two: 65 and 100 pad to 128 slots
    (cluster path, a second group of 64 lanes mostly padding), 257 pads to 512
    (the colour path above 256 slots).  The first, a middle and the last
    member match the oracle and the same member solved alone."""
    mesh, prob = _small_problem(precision=0, n_members=n_members, n_steps=6, dims=(4, 3, 2), ns=12, tol=1e-12)
    vs, gr = I.ensemble_members(95, n_members, I.CFG0_LAYERS["vs"])
    prob.vs = vs
    prob.gamma_ref = np.tile(gr[:, None], (1, 2))
    mh = gpu_ctx.mesh(mesh)
    out = gpu_ctx.solve(mh, mesh, prob)
    assert out["rc"] == 0 and out["vel"].shape[0] == n_members
    for m in (0, n_members // 2, n_members - 1):
        vref, _ = _oracle_vel(oracle_lib, mesh, prob, m)
        alone = gpu_ctx.solve(mh, mesh, prob, members=[m])
        e_or = oracle_lib.rel_l2(out["vel"][m], vref)
        e_al = oracle_lib.rel_l2(out["vel"][m], alone["vel"][0])
        say(n_members, "members: member", m, "vs oracle", e_or, "vs alone", e_al)
        assert np.abs(vref).max() > 0 and e_or < 1e-9 and e_al < 1e-12


def test_degenerate_inputs(gpu_ctx, oracle_lib, nlth_mod):
    """A one-cube mesh (6 tets, fewer than one cluster), FP64 and mixed, against
    the oracle; a record of zero input stays exactly at rest with no CG
    iterations; a problem of zero steps solves to empty results; stepping an
    ensemble past its record end does nothing."""
    for precision in (0, 1):
        mesh, prob = I.config(0, n_steps=8, mesh_dims=(1, 1, 1), n_members=2, cg_tol=1e-12, precision=precision,
                              n_springs=12)
        prob.input_acc = np.ascontiguousarray(prob.input_acc * 5.0)
        prob.input_acc[1] = 0.0  # member 1: no input
        mh = gpu_ctx.mesh(mesh)
        out = gpu_ctx.solve(mh, mesh, prob)
        assert out["rc"] == 0
        vref, _ = _oracle_vel(oracle_lib, mesh, prob, 0)
        err = oracle_lib.rel_l2(out["vel"][0], vref)
        say("one cube, precision", precision, "member 0 vs oracle", err)
        assert np.abs(vref).max() > 0 and err < 1e-9
        assert np.all(out["vel"][1] == 0.0) and np.all(out["iters"][1] == 0)
    mesh, prob = I.config(0, n_steps=4, mesh_dims=(2, 2, 1), n_members=1, cg_tol=1e-12, n_springs=12)
    out = gpu_ctx.solve(gpu_ctx.mesh(mesh), mesh, prob, n_steps=0)
    assert out["rc"] == 0 and out["vel"].size == 0
    mesh, prob = _small_problem(precision=0, n_steps=4, dims=(2, 2, 1), ns=12)
    mh = gpu_ctx.mesh(mesh)
    ens = gpu_ctx.ensemble(mh, mesh, prob)
    try:
        ens.step(4)
        first = ens.read()["vel"].copy()
        ens.step(3)  # past the end of the record
        assert ens.stats()["steps_done"] == 4 and np.array_equal(ens.read()["vel"], first)
    finally:
        ens.close()
