"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Tolerances:
  * stencil y = A x (FP64, same formula, different summation order): 1e-14 rel;
  * one source-transfer round with complex128 fronts: 1e-12 rel (direct solves of
    the local systems, condition numbers ~1e4);
  * the same with complex64 fronts: 2e-4 rel (FP32 rounding, 6e-8, times the
    local condition number and growth);
  * FGMRES solutions: 1e-10 rel-L2 (plain FP64 path at rel-res 1e-12) and 1e-8
    (complex64 fronts, FP64 outer iteration at rel-res 1e-10).
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


def _prm(w, **over):
    p = w.params()
    d = dict(nx=p["nx"], ny=p["ny"], k0=p["k0"], dx=p["dx"], dy=p["dy"], pml=p["pml"],
             pml_order=p["pml_order"], pml_R=p["pml_R"], px=p["px"], py=p["py"],
             overlap=p["overlap"], local_pml=p["local_pml"],
             local_pml_order=p["local_pml_order"], local_pml_R=p["local_pml_R"])
    d.update(over)
    return d


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


CASES = {
    "small": lambda: workloads.configs.small_random(nx=48, ny=40, pml=6, px=2, py=2, overlap=2,
                                                    local_pml=6, seed=3),
    "ragged": lambda: workloads.configs.small_random(nx=71, ny=53, pml=5, px=3, py=2, overlap=3,
                                                     local_pml=5, seed=4),
    "c1": lambda: workloads.configs.cylinder_tfsf(),
}


@pytest.mark.parametrize("case", list(CASES))
def test_stencil_matches_oracle(stf, ctx, case):
    w = CASES[case]()
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    x = workloads.sources.random_field(w.nx, w.ny, 11)
    y = pb.apply(x)
    assert _rel(y, A @ x.ravel()) < 1e-14


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("leaf", [0, 4, 64])
def test_round_c128_matches_oracle(stf, ctx, case, leaf):
    w = CASES[case]()
    pb = stf.Problem(ctx, _prm(w, leaf_size=leaf), w.eps_cells)
    assert pb.factor() is False
    B = ddm.SourceTransfer(w.params(), w.eps_cells)
    v = workloads.sources.random_field(w.nx, w.ny, 12)
    z = pb.precond(v)
    assert _rel(z, B.apply(v.ravel())) < 1e-12


@pytest.mark.parametrize("case", ["small", "c1"])
def test_round_c64_matches_oracle(stf, ctx, case):
    w = CASES[case]()
    pb = stf.Problem(ctx, _prm(w, front_prec=stf.STF_C64), w.eps_cells)
    pb.factor()
    B = ddm.SourceTransfer(w.params(), w.eps_cells)
    v = workloads.sources.random_field(w.nx, w.ny, 13)
    assert _rel(pb.precond(v), B.apply(v.ravel())) < 2e-4


# Degenerate shapes: the smallest grid (one front), strips four nodes wide,
# blocks without overlap, blocks only just wider than overlap + local PML;
# leaf_size 1 makes every separator a single node (the deepest trees).
DEGENERATE = {
    "3x3": dict(nx=3, ny=3, pml=0, px=1, py=1, overlap=0, local_pml=1),
    "strip_4x29": dict(nx=4, ny=29, pml=0, px=1, py=3, overlap=1, local_pml=2),
    "no_overlap_33x5": dict(nx=33, ny=5, pml=0, px=4, py=1, overlap=0, local_pml=1),
    "tight_6x6": dict(nx=6, ny=6, pml=0, px=2, py=2, overlap=1, local_pml=1),
}


@pytest.mark.parametrize("shape", list(DEGENERATE))
@pytest.mark.parametrize("leaf", [0, 1])
@pytest.mark.parametrize("prec,bar", [(0, 1e-12), (1, 2e-4)])
def test_round_degenerate_shapes_match_oracle(stf, ctx, shape, leaf, prec, bar):
    w = workloads.configs.small_random(seed=7, **DEGENERATE[shape])
    pb = stf.Problem(ctx, _prm(w, leaf_size=leaf, front_prec=prec), w.eps_cells)
    pb.factor()
    B = ddm.SourceTransfer(w.params(), w.eps_cells)
    v = workloads.sources.random_field(w.nx, w.ny, 14)
    assert _rel(pb.precond(v), B.apply(v.ravel())) < bar
    pb.close()


def test_single_subdomain_round_is_inverse(stf, ctx):
    w = workloads.configs.small_random(nx=40, ny=36, pml=6, px=1, py=1, seed=5)
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    pb.factor()
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    b = w.b[0]
    z = pb.precond(b)
    assert fdfd.relres(A, z.ravel(), b.ravel()) < 1e-13
    x, info = pb.solve(b, tol=1e-12)
    assert info[0]["iters"] == 1 and info[0]["relres_true"] < 1e-12


def test_stationary_algorithm1_matches_oracle(stf, ctx):
    """Algorithm 1 as the paper iterates it (x_0 = B b, x <- x + B (b - A x)),
    complex128 fronts on configuration 1: the relative residual of every round
    equals the oracle's (up to rounding, 1e-6 relative + 1e-12) and the 14th
    iterate equals the oracle's to 1e-10; tol 0 is never met (STF_ENOCONV)."""
    w = CASES["c1"]()
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    pb.factor()
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    B = ddm.SourceTransfer(w.params(), w.eps_cells)
    b = w.b[0]
    xr, hr = ddm.stationary(A, B, b.ravel(), 14)
    x, info = pb.stationary_solve(b, tol=0.0, max_rounds=14)
    assert info["rounds"] == 14 and info["status"] == 6
    h, hr = np.array(info["hist"]), np.array(hr)
    assert h.shape == hr.shape
    assert np.all(np.abs(h - hr) <= 1e-6 * hr + 1e-12)
    assert _rel(x, xr) < 1e-10
    pb.close()


def test_stationary_mixed_converges_to_direct_on_device(stf, ctx):
    """With complex64 fronts the rounds still drive the FP64 true residual down
    (each round corrects with the FP64 residual): tol 1e-10 is met, the field
    equals the direct solve to 1e-8; device tensors in and out."""
    import torch
    w = CASES["c1"]()
    pb = stf.Problem(ctx, _prm(w, front_prec=stf.STF_C64), w.eps_cells)
    pb.factor()
    b = w.b[0]
    bd = torch.from_numpy(b).cuda()
    x, info = pb.stationary_solve(bd, tol=1e-10, max_rounds=60)
    assert info["status"] == 0 and info["relres_true"] <= 1e-10
    assert info["rounds"] == len(info["hist"]) - 1
    h = info["hist"]
    assert all(b1 < b0 for b0, b1 in zip(h[:6], h[1:7]))
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    assert _rel(x.cpu().numpy(), fdfd.solve_direct(A, b.ravel()).reshape(b.shape)) < 1e-8
    pb.close()


def test_line_flux_matches_oracle(stf, ctx):
    """Power through grid lines (both axes, full and partial ranges, the first
    and last possible line) of a random field and of the configuration-1
    solution, against oracle/fdfd.line_flux (FP64, another summation order:
    1e-12 relative to the sum of the magnitudes); out-of-range lines are
    rejected."""
    w = CASES["ragged"]()
    p = w.params()
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    e = workloads.sources.random_field(w.nx, w.ny, 21)
    lines = [(1, 0, 0, w.nx), (1, w.ny - 2, 3, 40), (1, 20, 10, 10), (0, 0, 0, w.ny),
             (0, w.nx - 2, 5, w.ny), (0, 33, 7, 29)]
    for axis, index, lo, hi in lines:
        ref = fdfd.line_flux(e, w.nx, w.ny, axis, index, lo, hi, p["k0"], p["dx"], p["dy"])
        scale = fdfd.line_flux(np.abs(e), w.nx, w.ny, axis, index, lo, hi, p["k0"], p["dx"],
                               p["dy"]) + np.abs(e).max() ** 2 * max(hi - lo, 1) / p["k0"]
        got = pb.line_flux(e, axis, index, lo, hi)
        assert abs(got - ref) <= 1e-12 * scale, (axis, index, lo, hi, got, ref)
    for bad in [(2, 0, 0, 1), (1, w.ny - 1, 0, 1), (0, -1, 0, 1), (1, 0, 5, 4), (1, 0, 0, w.nx + 1)]:
        with pytest.raises(stf.StfError):
            pb.line_flux(e, *bad)
    pb.close()
    wc = CASES["c1"]()
    pc = wc.params()
    pb = stf.Problem(ctx, _prm(wc), wc.eps_cells)
    pb.factor()
    x, _ = pb.solve(wc.b[0], tol=1e-12)
    j = wc.ny // 2
    ref = fdfd.line_flux(x, wc.nx, wc.ny, 0, j, 20, wc.ny - 20, pc["k0"], pc["dx"], pc["dy"])
    assert pb.line_flux(x, 0, j, 20, wc.ny - 20) == pytest.approx(ref, rel=1e-12)
    import torch
    xd = torch.from_numpy(x).cuda()                 # the same field from device memory
    assert pb.line_flux(xd, 0, j, 20, wc.ny - 20) == pytest.approx(ref, rel=1e-12)
    pb.close()


def test_c1_solve_plain_fp64(stf, ctx):
    """Config 1 (plain method, complex128): FGMRES to rel-res 1e-12 equals the
    global direct solve to 1e-10."""
    w = workloads.configs.cylinder_tfsf()
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    pb.factor()
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    b = w.b[0]
    xref = fdfd.solve_direct(A, b.ravel())
    x, info = pb.solve(b, tol=1e-12, restart=30)
    assert info[0]["status"] == 0 and info[0]["iters"] <= 15
    assert _rel(x, xref) < 1e-10
    assert fdfd.relres(A, x.ravel(), b.ravel()) < 1e-12
    # The residual history starts at |b - A x0| / |b| = 1 and ends below tol.
    h = info[0]["history"]
    assert abs(h[0] - 1.0) < 1e-12 and h[-1] < 1e-12


def test_c1_solve_mixed_c64(stf, ctx):
    w = workloads.configs.cylinder_tfsf()
    pb = stf.Problem(ctx, _prm(w, front_prec=stf.STF_C64), w.eps_cells)
    pb.factor()
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    b = w.b[0]
    xref = fdfd.solve_direct(A, b.ravel())
    x, info = pb.solve(b, tol=1e-10, restart=30)
    assert info[0]["status"] == 0
    assert _rel(x, xref) < 1e-8


def test_device_buffers_and_multiple_rhs(stf, ctx):
    import torch
    w = workloads.configs.small_random(nx=64, ny=48, pml=6, px=2, py=2, overlap=2, local_pml=6,
                                       seed=6, nrhs=3)
    eps = torch.from_numpy(w.eps_cells).cuda()
    pb = stf.Problem(ctx, _prm(w), eps)
    pb.factor()
    bd = torch.from_numpy(w.b).cuda()
    xd, info = pb.solve(bd, tol=1e-12)
    torch.cuda.synchronize()
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    for r in range(3):
        xref = fdfd.solve_direct(A, w.b[r].ravel())
        assert _rel(xd[r].cpu().numpy(), xref) < 1e-10
        assert info[r]["status"] == 0


def test_user_initial_guess_resumes(stf, ctx):
    """A solve stopped early and resumed from its iterate (x0 = USER) reaches the
    same answer."""
    w = workloads.configs.small_random(nx=60, ny=50, pml=6, px=2, py=2, overlap=2, local_pml=6,
                                       seed=7)
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    pb.factor()
    b = w.b[0]
    x1, i1 = pb.solve(b, tol=1e-12, max_iter=2)
    assert i1[0]["status"] == 6      # STF_ENOCONV
    x2, i2 = pb.solve(b, tol=1e-12, x0=x1)
    assert abs(i2[0]["relres_x0"] - i1[0]["relres_true"]) < 1e-12
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    assert _rel(x2, fdfd.solve_direct(A, b.ravel())) < 1e-10


def test_errors(stf, ctx):
    w = workloads.configs.small_random(nx=40, ny=36, pml=6, px=2, py=2, overlap=2, local_pml=6)
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    with pytest.raises(stf.StfError) as e:
        pb.solve(w.b[0])
    assert e.value.status == 4           # STF_ESTATE: solve before factor
    pb.factor()
    bad = w.b[0].copy()
    bad[3, 4] = np.nan
    with pytest.raises(stf.StfError) as e:
        pb.solve(bad)
    assert e.value.status == 1           # STF_EINVAL: non-finite source
    cells = w.eps_cells.copy()
    cells[0, 0] = np.inf
    with pytest.raises(stf.StfError) as e:
        stf.Problem(ctx, _prm(w), cells)
    assert e.value.status == 1
    # Zero source: zero field, no iterations.
    x, info = pb.solve(np.zeros_like(w.b[0]))
    assert np.all(x == 0) and info[0]["iters"] == 0


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_rhs_equal_solo_solves(stf, ctx, prec):
    """Right-hand sides swept together (groups of up to four share every factor
    read) give exactly the solo solves: the per-RHS arithmetic is the same.
    Six RHS make a group of four and a group of two; one RHS is zero and one
    converges much later than the others (a scaled copy stops at the same
    iteration; a point source needs more), so RHS drop out of the lockstep at
    different iterations."""
    w = workloads.configs.small_random(nx=72, ny=60, pml=6, px=3, py=2, overlap=2, local_pml=6,
                                       seed=9, nrhs=4)
    b = np.concatenate([w.b, np.zeros((2,) + w.b.shape[1:], complex)])
    b[4] = 1e3 * w.b[0]
    b[5, 30, 36] = 1.0
    b[2] = 0.0
    pb = stf.Problem(ctx, _prm(w, front_prec=prec), w.eps_cells)
    pb.factor()
    tol = 1e-12 if prec == 0 else 1e-10
    xb, ib = pb.solve(b, tol=tol, restart=8)
    for r in range(6):
        xs, is_ = pb.solve(b[r], tol=tol, restart=8)
        assert ib[r]["iters"] == is_[0]["iters"] and ib[r]["restarts"] == is_[0]["restarts"]
        assert np.array_equal(xb[r], xs), r
        assert np.array_equal(ib[r]["history"], is_[0]["history"])
    assert ib[2]["iters"] == 0 and np.all(xb[2] == 0)
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    assert _rel(xb[5], fdfd.solve_direct(A, b[5].ravel())) < (1e-10 if prec == 0 else 1e-8)


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_round_equals_single_rounds(stf, ctx, prec):
    """The round swept for 1..4 vectors together equals the round of each vector
    alone, bit for bit (the sweeps share the factor reads, not the arithmetic)."""
    w = workloads.configs.small_random(nx=72, ny=60, pml=6, px=3, py=2, overlap=2, local_pml=6,
                                       seed=9, nrhs=4)
    pb = stf.Problem(ctx, _prm(w, front_prec=prec), w.eps_cells)
    pb.factor()
    v = np.concatenate([w.b, 1e3 * w.b[:1]])
    single = [pb.precond(v[r]) for r in range(5)]
    for k in range(1, 6):
        zb = pb.precond(v[:k])
        for r in range(k):
            assert np.array_equal(zb[r], single[r]), (k, r)


def test_stationary_eq20_stop_rule_matches_oracle(stf, ctx):
    """Algorithm 1 with the stop rule of Eq. (20): the overlap energies of the
    rounds follow the oracle's (1e-6 relative + 1e-12 of the first, complex128
    fronts), the iteration stops at the same round and the solution matches."""
    w = workloads.configs.cylinder_tfsf()
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    B = ddm.SourceTransfer(p, w.eps_cells)
    b = w.b[0]
    xr, er, hr = ddm.stationary_eq20(A, B, b.ravel(), 1e-8, 40)
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    pb.factor()
    x, info = pb.stationary_solve(b, tol=1e-8, max_rounds=40, stop="overlap")
    e = np.asarray(info["energy"])
    assert info["status"] == 0 and info["rounds"] == len(er) - 1
    assert np.all(np.abs(e - np.asarray(er)) <= 1e-6 * np.asarray(er) + 1e-12 * er[0])
    assert _rel(x, xr) < 1e-10
    # and the energies run down as Eq. (20) intends: below 1e-8 of the first
    assert e[-1] < 1e-8 * e[0]


def test_rcs_matches_oracle_and_mie(stf, ctx):
    """The near-to-far-field transform on the GPU against oracle.ntff (1e-11
    relative in F, same midpoint rule, another summation order), for the
    scattered-field solve of a dielectric cylinder (r = lambda/2, eps 4, 20
    points per wavelength, 2 x 2 subdomains): its RCS is within the
    discretisation error of the Mie series (as the oracle's is, 26% at 20 ppw),
    and a contour that does not enclose the scatterer sees (almost) nothing."""
    import math
    from oracle import ntff
    h, a, eps = 1.0 / 20, 0.5, 4.0
    L = 16
    n = int(round(2.5 / h)) + 2 * L
    c = (n - 1) / 2.0
    k0 = 2 * math.pi
    cells = workloads.geometry.cylinder(n, n, c * h, c * h, a, eps, dx=h, dy=h, subcells=16)
    p = dict(nx=n, ny=n, dx=h, dy=h, k0=k0, pml=(L,) * 4, pml_order=3, pml_R=1e-8, px=2, py=2,
             overlap=4, local_pml=12)
    X, Y = np.meshgrid(np.arange(n) * h - c * h, np.arange(n) * h - c * h)
    b = -k0 ** 2 * (fdfd.node_eps(cells) - 1) * np.exp(-1j * k0 * (X + c * h))
    pb = stf.Problem(ctx, p, cells)
    pb.factor()
    u, info = pb.solve(b, tol=1e-12, restart=30)
    m = L + 2
    box = (m, n - 1 - m, m, n - 1 - m)
    phis = np.linspace(0, 2 * math.pi, 72, endpoint=False)
    sig, F = pb.rcs(u, box, phis)
    Fr = ntff.far_field(u, h, h, box, k0, phis)
    assert np.linalg.norm(F - Fr) < 1e-11 * np.linalg.norm(Fr)
    ref = ntff.mie_rcs(k0, a, eps, phis)
    assert np.linalg.norm(sig - ref) < 0.35 * np.linalg.norm(ref)
    # a contour around empty space (left of the cylinder)
    sig0, _ = pb.rcs(u, (m, m + 10, n // 2 - 5, n // 2 + 5), phis)
    assert sig0.max() < 1e-3 * sig.max()
    with pytest.raises(stf.StfError):
        pb.rcs(u, (0, n - 1, 0, n - 1), phis)          # beyond the grid
    pb.close()
