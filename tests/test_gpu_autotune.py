"""Autotuner for the per-level launch shapes of the factorisation and of the
round's sweeps, through the C ABI.

* Every candidate shape of every level, and every subtree-sweep choice (level
  by level, or the deep levels one subtree per workgroup from each root depth
  that fits), gives the same round: the GPU round after forcing candidate i
  on every level (stf_tune_pick) against the oracle's round
  (oracle.ddm.SourceTransfer.apply), 1e-12 relative with complex128 fronts
  and 2e-4 with complex64 fronts, as for the built-in shapes.
* Every subtree choice and every launch shape of the stage levels of a staged
  order (rows, rows + columns, diagonal, two colours) gives the same sweep
  application: the GPU sweep after forcing choice i against the oracle's
  (oracle.ddm.sweep_apply), 1e-12 / 2e-4 as above; a batched diagonal solve after tuning its stages matches the direct
  solve.
* After stf_autotune a solve still meets its tolerance and matches the direct
  solve (oracle.fdfd.solve_direct): 1e-10 relative L2 at rel-res 1e-12
  (complex128), 1e-8 at rel-res 1e-10 (complex64); a batched solve after
  tuning the batch's own set as well.
* Tune files round-trip, and a file for another architecture or a malformed
  one is rejected without changing the context's entries.
"""
import numpy as np
import pytest

import workloads
from oracle import ddm, fdfd

pytestmark = pytest.mark.gpu


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
    # wavefront-kernel levels only
    "3x3_96": lambda: workloads.configs.small_random(nx=96, ny=96, pml=8, px=3, py=3, overlap=3,
                                                     local_pml=8, seed=12),
    # 2 x 2 subdomains of about 170^2 local nodes: every kernel kind (leaf LDS
    # factorisation, panel kernels, wavefront and workgroup sweeps in parts)
    "2x2_288": lambda: workloads.configs.small_random(nx=288, ny=288, pml=16, lam=20.0, px=2, py=2,
                                                      overlap=8, local_pml=16, seed=5),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec,bar", [(0, 1e-12), (1, 2e-4)])
def test_every_candidate_shape_gives_the_same_round(stf, ctx, case, prec, bar):
    w = CASES[case]()
    p = w.params()
    B = ddm.SourceTransfer(p, w.eps_cells)
    vs = np.stack([workloads.sources.random_field(w.nx, w.ny, 40 + s) for s in range(4)])
    refs = [B.apply(vs[s].ravel()) for s in range(4)]
    pb = stf.Problem(ctx, dict(p, front_prec=prec), w.eps_cells)
    try:
        for nr in (1, 4):
            most = ctx.tune_pick(pb, 0, nrhs=nr)
            assert most >= 2
            for idx in range(most):
                print("case %s prec %d nrhs %d candidate %d of %d" % (case, prec, nr, idx, most),
                      flush=True)
                ctx.tune_pick(pb, idx, nrhs=nr)
                pb.factor()
                if nr == 1:
                    z = pb.precond(vs[0])
                    assert _rel(z, refs[0]) < bar, idx
                else:
                    z = pb.precond(vs)
                    for s in range(4):
                        assert _rel(z[s], refs[s]) < bar, (idx, s)
    finally:
        ctx.tune_clear()
        pb.close()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("order", ["rows", "rows_cols", "diagonal", "checker"])
@pytest.mark.parametrize("prec,bar", [(0, 1e-12), (1, 2e-4)])
def test_every_staged_subtree_choice_gives_the_same_sweep(stf, ctx, case, order, prec, bar):
    w = CASES[case]()
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    B = ddm.SourceTransfer(p, w.eps_cells)
    v = workloads.sources.random_field(w.nx, w.ny, 23)
    ref = ddm.sweep_apply(B, A, v.ravel(), ddm.sweep_stages(B.subs, p["px"], p["py"], order))
    pb = stf.Problem(ctx, dict(p, front_prec=prec), w.eps_cells)
    try:
        pb.factor()
        ctx.tune_clear()
        most = ctx.tune_pick(pb, 0, nrhs=1, factor=False, sweeps=False, orders=(order,))
        assert most >= 2
        for idx in range(most):
            print("case %s order %s prec %d choice %d of %d" % (case, order, prec, idx, most),
                  flush=True)
            ctx.tune_pick(pb, idx, nrhs=1, factor=False, sweeps=False, orders=(order,))
            ops = [e[0][0] for e in ctx.tune_entries()]
            # the stage levels' shapes (operations 1, 2) and the stages' subtree choice
            assert [o for o in ops if o >= 3] == [3 + stf._abi.ORDERS[order]]
            assert set(ops) - {3 + stf._abi.ORDERS[order]} <= {1, 2}
            assert _rel(pb.sweep(v, order), ref) < bar, idx
    finally:
        ctx.tune_clear()
        pb.close()


def test_autotune_staged_then_batched_diagonal_solve(stf, ctx):
    import torch
    ws = [workloads.configs.disks_problem(k, sides=(64, 96, 128), pml=10, block=32, overlap=4,
                                          local_pml=8, nrhs=2, seed0=911) for k in range(3)]
    pbs = [stf.Problem(ctx, dict(w.params(), front_prec=1), w.eps_cells) for w in ws]
    try:
        ctx.tune_clear()
        rep = ctx.autotune(pbs, nrhs=2, reps=2, factor=True, sweeps=False, orders=("diagonal",))
        print("autotune report", rep, flush=True)
        ent = ctx.tune_entries()
        st = [e for e in ent if e[0][0] == 3 + stf._abi.ORDERS["diagonal"]]
        assert len(st) == 1 and st[0][0][2] == 2 and st[0][2][0] <= st[0][2][1]
        xs, infos = stf.batch_solve(ctx, pbs, [torch.from_numpy(w.b).cuda() for w in ws], tol=1e-10,
                                    restart=12, max_iter=400, order="diagonal")
        for p, w in enumerate(ws):
            A = fdfd.global_matrix(w.params(), w.eps_cells)
            for r in range(w.b.shape[0]):
                assert infos[p][r]["status"] == 0 and infos[p][r]["relres_true"] <= 1e-10
                assert _rel(xs[p][r].cpu().numpy(), fdfd.solve_direct(A, w.b[r].ravel())) < 1e-8
    finally:
        ctx.tune_clear()
        for pb in pbs:
            pb.close()


@pytest.mark.parametrize("prec,tol,bar", [(0, 1e-12, 1e-10), (1, 1e-10, 1e-8)])
def test_autotune_then_solve_matches_direct(stf, ctx, prec, tol, bar):
    w = CASES["2x2_288"]()
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    ref = fdfd.solve_direct(A, w.b[0].ravel())
    pb = stf.Problem(ctx, dict(p, front_prec=prec), w.eps_cells)
    try:
        ctx.tune_clear()
        rep = ctx.autotune(pb, nrhs=1, reps=2)
        levels = stf.plan_query(dict(p, front_prec=prec))["max_depth"] + 1
        print("autotune report", rep, flush=True)
        assert rep["levels"] == 3 * levels               # factorisation, forward and backward sweeps
        ent = ctx.tune_entries()
        assert len([e for e in ent if e[0][0] <= 2]) == 3 * levels
        fuse = [e for e in ent if e[0][0] == 3]             # the subtree choice of the problem
        assert len(fuse) == 1 and fuse[0][1][1] == rep["fuse_depth"]
        assert 0.0 < rep["ms_tuned"] <= rep["ms_default"]
        assert 0.0 < rep["ms_round_tuned"] <= rep["ms_round_default"]
        for key, shape, ms in ent:
            assert key[1] == (8 if prec else 16) and shape[0] in (1, 2) and ms[0] <= ms[1]
        x, info = pb.solve(w.b[0], tol=tol, restart=30, max_iter=400)
        assert info[0]["status"] == 0 and info[0]["relres_true"] <= tol
        assert _rel(x, ref) < bar
    finally:
        ctx.tune_clear()
        pb.close()


def test_batch_autotune_then_batch_solve(stf, ctx):
    import torch
    ws = [workloads.configs.disks_problem(k, sides=(64, 96, 128), pml=10, block=32, overlap=4,
                                          local_pml=8, nrhs=2, seed0=908) for k in range(3)]
    refs = []
    for w in ws:
        A = fdfd.global_matrix(w.params(), w.eps_cells)
        refs.append([fdfd.solve_direct(A, w.b[r].ravel()) for r in range(w.b.shape[0])])
    pbs = [stf.Problem(ctx, dict(w.params(), front_prec=1), w.eps_cells) for w in ws]
    try:
        ctx.tune_clear()
        rep = ctx.autotune(pbs, nrhs=2, reps=2)
        assert rep["levels"] > 0
        bs = [torch.from_numpy(w.b).cuda() for w in ws]
        xs, infos = stf.batch_solve(ctx, pbs, bs, tol=1e-10, restart=12, max_iter=400)
        for p, w in enumerate(ws):
            for r in range(w.b.shape[0]):
                assert infos[p][r]["status"] == 0 and infos[p][r]["relres_true"] <= 1e-10
                assert _rel(xs[p][r].cpu().numpy(), refs[p][r]) < 1e-8, (p, r)
    finally:
        ctx.tune_clear()
        for pb in pbs:
            pb.close()


def test_tune_file_round_trip_and_rejects(stf, ctx, tmp_path):
    w = CASES["3x3_96"]()
    pb = stf.Problem(ctx, dict(w.params(), front_prec=1), w.eps_cells)
    try:
        ctx.tune_clear()
        ctx.autotune(pb, nrhs=4, reps=1)
        ent = ctx.tune_entries()
        assert ent
        path = tmp_path / "tune.txt"
        ctx.tune_save(str(path))
        ctx.tune_clear()
        assert ctx.tune_entries() == []
        ctx.tune_load(str(path))
        got = ctx.tune_entries()
        assert [(k, s) for k, s, _ in got] == [(k, s) for k, s, _ in ent]
        for (_, _, a), (_, _, b) in zip(got, ent):
            assert np.allclose(a, b, rtol=1e-6)
        lines = path.read_text().splitlines()
        head = lines[0].split()
        assert head[0] == "stfdfd-tune" and head[1] == "1" and int(head[3]) == len(ent)
        other = tmp_path / "other.txt"
        other.write_text("\n".join([" ".join(head[:2] + ["gfx000"] + head[3:])] + lines[1:]) + "\n")
        with pytest.raises(stf.StfError) as e:
            ctx.tune_load(str(other))
        assert e.value.status == 1 and "gfx000" in str(e.value)
        bad = tmp_path / "bad.txt"
        bad.write_text(lines[0] + "\n" + "0 8 0 1 1\n")
        with pytest.raises(stf.StfError):
            ctx.tune_load(str(bad))
        assert [(k, s) for k, s, _ in ctx.tune_entries()] == [(k, s) for k, s, _ in ent]
        # a solve with the loaded shapes
        pb.factor()
        x, info = pb.solve(w.b[0], tol=1e-10, restart=30, max_iter=400)
        assert info[0]["status"] == 0
    finally:
        ctx.tune_clear()
        pb.close()
