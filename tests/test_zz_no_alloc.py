"""The allocation-free round (stf_precond_apply_noalloc) against the allocating
one (stf_precond_apply), through the C ABI: the same kernels on the same inputs,
so the outputs must be identical; two calls in a row, the second on a smaller
problem (the static workspace keeps the first call's contents), plus the size
limit and the state check."""
import numpy as np
import pytest

import workloads
from oracle import ddm

pytestmark = pytest.mark.gpu


def _prm(w, **over):
    d = dict(w.params())
    d.update(over)
    return d


def test_noalloc_round_equals_allocating_round_on_two_calls():
    import torch
    import paper_2509_20801_amd as stf
    ctx = stf.Context(0)
    cases = [(workloads.configs.small_random(nx=300, ny=260, pml=12, px=3, py=3, overlap=4,
                                             local_pml=8, seed=31), stf.STF_C64),
             (workloads.configs.small_random(nx=71, ny=53, pml=5, px=3, py=2, overlap=3,
                                             local_pml=5, seed=4), stf.STF_C128)]
    for w, prec in cases:
        print("noalloc case %dx%d prec=%d" % (w.nx, w.ny, prec), flush=True)
        pb = stf.Problem(ctx, _prm(w, front_prec=prec), w.eps_cells)
        pb.factor()
        v = torch.from_numpy(workloads.sources.random_field(w.nx, w.ny, 41)).cuda()
        z_ref = pb.precond(v)
        z = torch.full_like(v, complex("nan"))
        pb.precond_noalloc(v, z)
        torch.cuda.synchronize()
        assert torch.equal(z, z_ref)
        # and the round itself against the oracle (complex128: 1e-12, complex64: 2e-4)
        B = ddm.SourceTransfer(w.params(), w.eps_cells)
        zr = B.apply(v.cpu().numpy().ravel())
        err = np.linalg.norm(z.cpu().numpy().ravel() - zr) / np.linalg.norm(zr)
        assert err < (2e-4 if prec == stf.STF_C64 else 1e-12)
        pb.close()
    ctx.close()


def test_noalloc_round_rejects_oversized_and_unfactored_problems():
    import torch
    import paper_2509_20801_amd as stf
    ctx = stf.Context(0)
    # 1200^2 with complex128 fronts needs ~145 MB of workspace (> 128 MiB): rejected
    # before any launch (the problem is not even factored).
    w = workloads.configs.small_random(nx=1200, ny=1200, pml=20, px=8, py=8, overlap=8,
                                       local_pml=16, seed=2)
    pb = stf.Problem(ctx, _prm(w, front_prec=stf.STF_C128), w.eps_cells)
    v = torch.zeros((w.ny, w.nx), dtype=torch.complex128, device="cuda")
    z = torch.empty_like(v)
    with pytest.raises(stf.StfError) as e:
        pb.precond_noalloc(v, z)
    assert e.value.status == 1 and "at most" in str(e.value)
    pb.close()
    w = workloads.configs.small_random(nx=48, ny=40, pml=6, px=2, py=2, overlap=2, local_pml=6,
                                       seed=3)
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    v = torch.zeros((w.ny, w.nx), dtype=torch.complex128, device="cuda")
    with pytest.raises(stf.StfError) as e:
        pb.precond_noalloc(v, torch.empty_like(v))
    assert e.value.status == 4
    pb.close()
    ctx.close()
