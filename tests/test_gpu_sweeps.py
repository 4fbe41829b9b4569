"""Staged (multiplicative) source-transfer orders on the GPU against the oracle
(oracle.ddm.sweep_stages / sweep_apply), through the C ABI.  One application:
1e-12 relative with complex128 fronts (direct local solves), 2e-4 with
complex64 fronts, as for the Jacobi round.  FGMRES with a staged order: 1e-10
relative L2 at rel-res 1e-12 (complex128), 1e-8 at rel-res 1e-10 (complex64)."""
import numpy as np
import pytest

import workloads
from oracle import ddm, fdfd

pytestmark = pytest.mark.gpu

ORDERS = ["rows", "rows_cols", "diagonal", "checker"]


@pytest.fixture(scope="module")
def stf():
    import paper_2509_20801_amd as stf
    return stf


@pytest.fixture(scope="module")
def ctx(stf):
    return stf.Context(0)


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


CASES = {
    "2x2": lambda: workloads.configs.small_random(nx=48, ny=40, pml=6, px=2, py=2, overlap=2,
                                                  local_pml=6, seed=3),
    "ragged_3x2": lambda: workloads.configs.small_random(nx=71, ny=53, pml=5, px=3, py=2, overlap=3,
                                                         local_pml=5, seed=4),
    "3x3": lambda: workloads.configs.small_random(nx=96, ny=96, pml=8, px=3, py=3, overlap=3,
                                                  local_pml=8, seed=12),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("prec,bar", [(0, 1e-12), (1, 2e-4)])
def test_sweep_application_matches_oracle(stf, ctx, case, order, prec, bar):
    w = CASES[case]()
    p = w.params()
    pb = stf.Problem(ctx, dict(p, front_prec=prec), w.eps_cells)
    pb.factor()
    A = fdfd.global_matrix(p, w.eps_cells)
    B = ddm.SourceTransfer(p, w.eps_cells)
    v = workloads.sources.random_field(w.nx, w.ny, 17)
    ref = ddm.sweep_apply(B, A, v.ravel(), ddm.sweep_stages(B.subs, p["px"], p["py"], order))
    assert _rel(pb.sweep(v, order), ref) < bar
    pb.close()


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("prec,tol,bar", [(0, 1e-12, 1e-10), (1, 1e-10, 1e-8)])
def test_fgmres_with_staged_order_matches_direct(stf, ctx, order, prec, tol, bar):
    w = CASES["3x3"]()
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    xref = fdfd.solve_direct(A, w.b[0].ravel())
    pb = stf.Problem(ctx, dict(p, front_prec=prec), w.eps_cells)
    pb.factor()
    x, info = pb.solve(w.b[0], tol=tol, restart=30, order=order)
    _, add = pb.solve(w.b[0], tol=tol, restart=30)
    assert info[0]["status"] == 0 and info[0]["relres_true"] <= tol
    assert _rel(x, xref) < bar
    assert info[0]["iters"] < add[0]["iters"]
    pb.close()


def test_batched_solve_with_diagonal_sweeps(stf, ctx):
    """A batch of disk problems (2x2 to 4x4 subdomains, 1-4 right-hand sides) in
    the four-diagonal order: stage t of every problem in the same launches."""
    import torch
    ws = [workloads.configs.disks_problem(k, sides=(64, 96, 128), pml=10, block=32, overlap=4,
                                          local_pml=8, nrhs=(1, 4, 2, 3)[k % 4], seed0=908)
          for k in range(5)]
    pbs = [stf.Problem(ctx, dict(w.params(), front_prec=1), w.eps_cells) for w in ws]
    xs, infos = stf.batch_solve(ctx, pbs, [torch.from_numpy(w.b).cuda() for w in ws], tol=1e-10,
                                restart=12, order="diagonal")
    _, add = stf.batch_solve(ctx, pbs, [torch.from_numpy(w.b).cuda() for w in ws], tol=1e-10,
                             restart=12)
    for p, w in enumerate(ws):
        A = fdfd.global_matrix(w.params(), w.eps_cells)
        for r in range(w.b.shape[0]):
            assert infos[p][r]["status"] == 0
            assert _rel(xs[p][r].cpu().numpy(), fdfd.solve_direct(A, w.b[r].ravel())) < 1e-8
            assert infos[p][r]["iters"] < add[p][r]["iters"] or w.px == 1
    for pb in pbs:
        pb.close()
