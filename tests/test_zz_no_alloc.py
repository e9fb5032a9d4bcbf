"""The allocation-free operator application (for callers that cannot
allocate device memory) on device buffers, against nlth_apply_operator (same
kernels: bitwise equal) and the oracle's assembled matrices (1e-13), on two
calls in a row, the second with a smaller mesh; a mesh beyond the scratch
array's capacity is refused."""
import numpy as np
import pytest

from paper_2604_02755_amd import inputs as I

pytestmark = pytest.mark.gpu


def _rand_D(rng, ne, G0=4e7, lam=3e8):
    base = np.zeros((6, 6))
    base[:3, :3] = lam
    base[np.arange(3), np.arange(3)] += 2 * G0
    base[3:, 3:] = np.eye(3) * G0
    L = rng.normal(size=(ne, 4, 6, 6)) * 0.3 * G0 ** 0.5
    D = base + np.einsum("eiab,eicb->eiac", L, L)
    iu = np.triu_indices(6)
    return np.ascontiguousarray(D[:, :, iu[0], iu[1]])


def test_noalloc_apply_matches_apply_operator_and_oracle(nlth_mod, oracle_lib):
    import torch
    dev = torch.device("cuda", 0)
    ctx = nlth_mod.Context(0, use_torch_stream=True)
    try:
        rng = np.random.default_rng(5)
        for dims in ((6, 5, 4), (4, 3, 2)):  # the second call has the smaller input
            mesh, prob = I.config(0, n_steps=1, mesh_dims=dims)
            mh = ctx.mesh(mesh)
            D = _rand_D(rng, mesh.n_tets)
            h = rng.uniform(0, 0.2, mesh.n_tets)
            x = rng.normal(size=mesh.n_dof)
            Dt = torch.from_numpy(D).to(dev)
            ht = torch.from_numpy(h).to(dev)
            xt = torch.from_numpy(x).to(dev)
            for which in (0, 1, 2):
                yt = torch.full((mesh.n_dof,), float("nan"), dtype=torch.float64, device=dev)
                torch.cuda.synchronize()
                print("no-alloc apply", dims, "op", which, flush=True)
                nlth_mod.nlth_apply_operator_noalloc(ctx.h, mh, prob, which, Dt.data_ptr(), ht.data_ptr(),
                                                     xt.data_ptr(), yt.data_ptr())
                torch.cuda.synchronize()
                y = yt.cpu().numpy()
                y_ref = ctx.apply_operator(mh, prob, which, 0, D, h, x)
                y_or = oracle_lib.apply_operator(mesh, prob, which, D, h, x)
                err = np.linalg.norm(y - y_or) / np.linalg.norm(y_or)
                print("  equal to nlth_apply_operator:", bool(np.array_equal(y, y_ref)), "rel err vs oracle", err,
                      flush=True)
                assert np.array_equal(y, y_ref)
                assert err < 1e-13
            # h = NULL means zero element damping
            yt = torch.empty((mesh.n_dof,), dtype=torch.float64, device=dev)
            nlth_mod.nlth_apply_operator_noalloc(ctx.h, mh, prob, 0, Dt.data_ptr(), 0, xt.data_ptr(), yt.data_ptr())
            torch.cuda.synchronize()
            y0 = ctx.apply_operator(mh, prob, 0, 0, D, None, x)
            assert np.array_equal(yt.cpu().numpy(), y0)
        # beyond the scratch array: refused before any launch
        big, pb = I.config(0, n_steps=1, mesh_dims=(24, 24, 20))
        mb = ctx.mesh(big)
        Db = torch.zeros((big.n_tets, 4, 21), dtype=torch.float64, device=dev)
        xb = torch.zeros(big.n_dof, dtype=torch.float64, device=dev)
        yb = torch.zeros(big.n_dof, dtype=torch.float64, device=dev)
        with pytest.raises(nlth_mod.NlthError) as ei:
            nlth_mod.nlth_apply_operator_noalloc(ctx.h, mb, pb, 0, Db.data_ptr(), 0, xb.data_ptr(), yb.data_ptr())
        print("large mesh refused:", str(ei.value), flush=True)
        assert ei.value.code == nlth_mod.NLTH_EINVAL and "scratch" in str(ei.value)
    finally:
        torch.cuda.synchronize()
        ctx.close()
