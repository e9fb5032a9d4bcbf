"""State paging (Section 2.2, Algorithm 3): the per-spring law state lives in
pinned host memory and is streamed through a ring of device chunks on copy
streams.  With an HBM budget too small for the state, every member matches
the oracle (tolerance 1e-12 on both sides, 1e-9 relative L2 on receiver
velocity), and the results are bitwise identical to the resident run (same
kernels, same order).  The pinned host copy holds exactly the law state:
4 points x N_s springs x 36 B per element and member slot (the paper's four
doubles and two flags, with both flags in one int32).  By default a paged
ensemble runs as two member sets whose solves alternate with each other's law
phases, so that the transfers overlap a solve; one set is a context option."""
import sys

import numpy as np
import pytest

from paper_2604_02755_amd import inputs as I

pytestmark = pytest.mark.gpu


def _problem():
    mesh, prob = I.config(0, n_steps=12, mesh_dims=(5, 4, 3), n_members=3, cg_tol=1e-12,
                          precision=I.PRECISION_MIXED)
    vs, gr = I.ensemble_members(55, 3, I.CFG0_LAYERS["vs"])
    prob.vs = vs
    prob.gamma_ref = np.tile(gr[:, None], (1, 2))
    prob.input_acc = 5.0 * I.member_waves(0, range(3), prob.n_steps, prob.dt)
    return mesh, prob


def _oracle_check(oracle_lib, mesh, prob, out, what):
    for m in range(prob.n_members):
        ref = oracle_lib.run(mesh, prob, member=m)
        err = oracle_lib.rel_l2(out["vel"][m], ref["vel"])
        print(f"  {what}: member {m} rel L2 vs oracle {err:.3e}", flush=True)
        assert np.abs(ref["vel"]).max() > 0 and err < 1e-9


def test_paged_state_matches_oracle_and_resident(nlth_mod, oracle_lib):
    mesh, prob = _problem()
    outs, stats = [], []
    for budget in (0, 24 << 20):  # default budget, then 24 MiB (the state alone is ~35 MB)
        print("paging case: hbm budget", budget, "one member set", flush=True)
        ctx = nlth_mod.Context(0, hbm_budget=budget, use_torch_stream=False, paging_sets=1)
        try:
            mh = ctx.mesh(mesh)
            ens = ctx.ensemble(mh, mesh, prob)
            ens.step(prob.n_steps)
            outs.append(ens.read())
            stats.append(ens.stats())
            ens.close()
        finally:
            ctx.close()
    print("  paged flags", stats[0]["paged"], stats[1]["paged"], "h2d bytes", stats[1]["h2d_bytes"],
          "d2h bytes", stats[1]["d2h_bytes"], flush=True)
    assert stats[0]["paged"] == 0 and stats[1]["paged"] == 1
    assert stats[1]["h2d_bytes"] > 0 and stats[1]["d2h_bytes"] > 0
    # pinned host bytes = the law state: elements (padded to the layout's
    # element blocks) x 4 points x springs x member slots x 36 B
    MB = stats[1]["members_padded"]
    EB = max(1, 64 // MB)
    ne_pad = -(-mesh.n_tets // EB) * EB
    want = ne_pad * 4 * prob.n_springs * MB * 36
    print("  host bytes", stats[1]["host_bytes"], "expected", want, flush=True)
    assert stats[1]["host_bytes"] == want
    _oracle_check(oracle_lib, mesh, prob, outs[1], "paged")
    assert np.array_equal(outs[0]["vel"], outs[1]["vel"])
    assert np.array_equal(outs[0]["iters"], outs[1]["iters"])
    assert np.abs(outs[0]["vel"]).max() > 0


def test_zero_copy_law_matches_oracle_and_resident(nlth_mod, oracle_lib):
    """The ablation of the pipeline (the law kernel working on the pinned host
    state over the host link) computes the same thing: every member matches
    the oracle and the run is bitwise equal to the resident one, also when it
    alternates with the pipelined copies; a resident ensemble refuses it."""
    mesh, prob = _problem()
    outs = []
    for budget, plan in ((0, None), (24 << 20, (1, 0, 1))):
        print("zero-copy case: hbm budget", budget, "plan", plan, flush=True)
        ctx = nlth_mod.Context(0, hbm_budget=budget, use_torch_stream=False, paging_sets=1)
        try:
            mh = ctx.mesh(mesh)
            ens = ctx.ensemble(mh, mesh, prob)
            if plan is None:
                with pytest.raises(nlth_mod.NlthError) as ei:
                    ens.set_tuning(zero_copy=1)
                assert ei.value.code == nlth_mod.NLTH_EINVAL
                ens.step(prob.n_steps)
            else:
                for zc in plan:  # zero-copy, pipelined, zero-copy: 4 steps each
                    ens.set_tuning(zero_copy=zc)
                    ens.step(prob.n_steps // len(plan))
                assert ens.stats()["paged"] == 1
            outs.append(ens.read())
            ens.close()
        finally:
            ctx.close()
    _oracle_check(oracle_lib, mesh, prob, outs[1], "zero-copy")
    assert np.array_equal(outs[0]["vel"], outs[1]["vel"])
    assert np.array_equal(outs[0]["iters"], outs[1]["iters"])
    assert np.abs(outs[0]["vel"]).max() > 0


def test_two_member_sets_match_oracle(nlth_mod, oracle_lib):
    """The paged ensemble as two member sets (members 0-1 and 2),
    each on its own compute stream, sharing the transfer-in stream.  Every member
    matches the oracle and the one-set paged run (1e-12 relative: the sets pad
    to other member-slot counts, which changes only the grouping of the dot
    products' partial sums), the members keep their numbering and iteration
    counts, the pinned host copy is the two sets' law state, and the
    zero-copy ablation works on both sets."""
    mesh, prob = _problem()
    outs, stats = [], []
    for sets, zc in ((1, 0), (2, 0), (2, 1)):
        print("member sets", sets, "zero-copy", zc, flush=True)
        ctx = nlth_mod.Context(0, hbm_budget=24 << 20, use_torch_stream=False, paging_sets=sets)
        try:
            mh = ctx.mesh(mesh)
            ens = ctx.ensemble(mh, mesh, prob)
            if zc:
                ens.set_tuning(zero_copy=1)
            ens.step(5)
            ens.step(prob.n_steps - 5)
            outs.append(ens.read())
            stats.append(ens.stats())
            ens.close()
        finally:
            ctx.close()
    for st in stats:
        print("  sets", st["member_sets"], "paged", st["paged"], "members", st["n_members"], "slots",
              st["members_padded"], "host bytes", st["host_bytes"], "h2d", st["h2d_bytes"], flush=True)
    assert [st["member_sets"] for st in stats] == [1, 2, 2]
    assert all(st["paged"] == 1 and st["n_members"] == 3 and st["steps_done"] == prob.n_steps for st in stats)
    # sets of 2 and 1 members: slots 2 and 1, element blocks of 32 and 64
    want = sum(-(-mesh.n_tets // (64 // mb)) * (64 // mb) * 4 * prob.n_springs * mb * 36 for mb in (2, 1))
    assert stats[1]["members_padded"] == 3 and stats[1]["host_bytes"] == want
    assert stats[1]["h2d_bytes"] > 0 and stats[2]["h2d_bytes"] >= 0
    _oracle_check(oracle_lib, mesh, prob, outs[1], "two sets")
    for o in outs[1:]:
        for m in range(prob.n_members):
            err = oracle_lib.rel_l2(o["vel"][m], outs[0]["vel"][m])
            assert err < 1e-12, (m, err)
        assert np.max(np.abs(o["iters"][:, :, 0] - outs[0]["iters"][:, :, 0])) <= 1
    assert np.array_equal(outs[1]["vel"], outs[2]["vel"])
