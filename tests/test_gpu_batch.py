"""Batched solve (stf_batch_solve) through the C ABI: several problems of the
disk workload at reduced size (interior sides 64-128, 2x2 to 4x4 subdomains),
1 to 4 right-hand sides each, factored together and solved by one lockstep
FGMRES.  Every system is checked against the FP64 oracle's direct solve
(1e-10 relative L2 at rel-res 1e-12 with complex128 fronts, 1e-8 at rel-res
1e-10 with complex64 fronts) and against its solo solve (within the sum of
both tolerances' error); the HIP-graph replay of a cycle is checked against
the same cycles launched one kernel at a time (identical results)."""
import os

import numpy as np
import pytest

import workloads
from oracle import fdfd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stf():
    import paper_2509_20801_amd as stf
    return stf


@pytest.fixture(scope="module")
def ctx(stf):
    return stf.Context(0)


def _small_batch(count=6, nrhs=(1, 4, 2, 3, 4, 1)):
    ws = []
    for k in range(count):
        w = workloads.configs.disks_problem(k, sides=(64, 96, 128), pml=10, block=32, overlap=4,
                                            local_pml=8, nrhs=nrhs[k % len(nrhs)], seed0=908)
        ws.append(w)
    return ws


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.fixture(scope="module")
def batch():
    ws = _small_batch()
    refs = []
    for w in ws:
        A = fdfd.global_matrix(w.params(), w.eps_cells)
        refs.append([fdfd.solve_direct(A, w.b[r].ravel()) for r in range(w.b.shape[0])])
    return ws, refs


@pytest.mark.parametrize("prec,tol,bar", [(0, 1e-12, 1e-10), (1, 1e-10, 1e-8)])
def test_batch_matches_oracle_and_solo(stf, ctx, batch, prec, tol, bar):
    import torch
    ws, refs = batch
    print("batch of %d problems, sides %s, prec %d" % (len(ws), [w.nx for w in ws], prec), flush=True)
    pbs = [stf.Problem(ctx, dict(w.params(), front_prec=prec), w.eps_cells) for w in ws]
    bs = [torch.from_numpy(w.b).cuda() for w in ws]
    xs, infos = stf.batch_solve(ctx, pbs, bs, tol=tol, restart=12, max_iter=400)
    for p, w in enumerate(ws):
        pbs[p].factor()
        xsolo, isolo = pbs[p].solve(w.b, tol=tol, restart=12, max_iter=400)
        for r in range(w.b.shape[0]):
            inf = infos[p][r]
            assert inf["status"] == 0 and inf["relres_true"] <= tol, (p, r, inf)
            xr = xs[p][r].cpu().numpy()
            assert _rel(xr, refs[p][r]) < bar, (p, r)
            assert _rel(xr, xsolo[r]) < 2 * bar, (p, r)
            # same preconditioner and method: iteration counts as in the solo solve
            assert abs(inf["iters"] - isolo[r]["iters"]) <= 2, (p, r, inf["iters"], isolo[r]["iters"])
            assert inf["t_factor_ms"] > 0 and inf["t_solve_ms"] > 0
            assert len(inf["history"]) == inf["iters"] + 1
    for pb in pbs:
        pb.close()


def test_batch_graph_replays_equal_eager_launches(stf, ctx, batch, monkeypatch):
    """Several cycles (restart 4) so that the captured graph is replayed many
    times, with host reads and eager work between the replays; every replay's
    result equals the kernel-by-kernel launches bit for bit."""
    import torch
    ws, refs = batch
    pbs = [stf.Problem(ctx, dict(w.params(), front_prec=1), w.eps_cells) for w in ws]
    bs = [torch.from_numpy(w.b).cuda() for w in ws]
    monkeypatch.delenv("STF_BATCH_EAGER", raising=False)
    xg, ig = stf.batch_solve(ctx, pbs, bs, tol=1e-10, restart=4, max_iter=400)
    xg2, ig2 = stf.batch_solve(ctx, pbs, bs, tol=1e-10, restart=4, max_iter=400)
    monkeypatch.setenv("STF_BATCH_EAGER", "1")
    xe, ie = stf.batch_solve(ctx, pbs, bs, tol=1e-10, restart=4, max_iter=400)
    monkeypatch.delenv("STF_BATCH_EAGER")
    for p in range(len(ws)):
        assert max(i["restarts"] for i in ig[p]) >= 2
        assert torch.equal(xg[p], xe[p]) and torch.equal(xg2[p], xe[p]), p
        assert [i["iters"] for i in ig[p]] == [i["iters"] for i in ie[p]]
    for pb in pbs:
        pb.close()


def test_batch_with_kernel_timing_on(stf, ctx, batch, monkeypatch):
    """Per-kernel timing on during a batched solve: the kernels the cycle's
    graph captures are launched plainly (a timer declines during capture), the
    eager launches carry their dispatch events, and both runs equal the untimed
    ones bit for bit; the factorisation's kernels are timed."""
    import torch
    ws, refs = batch
    pbs = [stf.Problem(ctx, dict(w.params(), front_prec=1), w.eps_cells) for w in ws]
    bs = [torch.from_numpy(w.b).cuda() for w in ws]
    monkeypatch.delenv("STF_BATCH_EAGER", raising=False)
    x0, i0 = stf.batch_solve(ctx, pbs, bs, tol=1e-10, restart=4, max_iter=400)
    lu0 = ctx.kernel_stats("front_lu")
    ctx.set_timing(True)
    try:
        xg, ig = stf.batch_solve(ctx, pbs, bs, tol=1e-10, restart=4, max_iter=400)
        lu1 = ctx.kernel_stats("front_lu")
        monkeypatch.setenv("STF_BATCH_EAGER", "1")
        xe, ie = stf.batch_solve(ctx, pbs, bs, tol=1e-10, restart=4, max_iter=400)
    finally:
        ctx.set_timing(False)
        monkeypatch.delenv("STF_BATCH_EAGER", raising=False)
    assert lu1[1] > lu0[1] and lu1[0] > lu0[0]
    for p in range(len(ws)):
        assert torch.equal(xg[p], x0[p]) and torch.equal(xe[p], x0[p]), p
        assert [i["iters"] for i in ig[p]] == [i["iters"] for i in i0[p]]
    for pb in pbs:
        pb.close()


def test_batch_host_buffers_and_user_guess(stf, ctx, batch):
    ws, refs = batch
    ws, refs = ws[:3], refs[:3]
    pbs = [stf.Problem(ctx, dict(w.params(), front_prec=0), w.eps_cells) for w in ws]
    xs, infos = stf.batch_solve(ctx, pbs, [w.b for w in ws], tol=1e-6, restart=8)
    # resume from the loose solution: fewer iterations to the tight tolerance
    xt, it2 = stf.batch_solve(ctx, pbs, [w.b for w in ws], tol=1e-12, restart=8, x0=xs)
    for p, w in enumerate(ws):
        for r in range(w.b.shape[0]):
            assert _rel(xt[p][r], refs[p][r]) < 1e-10
            assert it2[p][r]["relres_x0"] <= 1e-6
    for pb in pbs:
        pb.close()


def test_batch_rejects_invalid_batches(stf, ctx, batch):
    ws, _ = batch
    a = stf.Problem(ctx, dict(ws[0].params(), front_prec=0), ws[0].eps_cells)
    b = stf.Problem(ctx, dict(ws[1].params(), front_prec=1), ws[1].eps_cells)
    with pytest.raises(stf.StfError) as e:
        stf.batch_solve(ctx, [a, b], [ws[0].b, ws[1].b])
    assert e.value.status == 1                       # mixed front precisions
    with pytest.raises(stf.StfError) as e:
        stf.batch_solve(ctx, [a, a], [ws[0].b, ws[0].b])
    assert e.value.status == 1                       # the same problem twice
    with pytest.raises(stf.StfError) as e:
        stf.batch_solve(ctx, [a], [ws[0].b], restart=40)
    assert e.value.status == 1                       # restart beyond the batched limit
    a.close()
    b.close()
