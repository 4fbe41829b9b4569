"""Pins for the oracle's overlapping decomposition and source-transfer round
(Sec. 2.3, Eqs. (14)-(21), Algorithm 1).  CPU only."""
import numpy as np
import pytest

import workloads
from oracle import ddm, fdfd, krylov


def _setup(w):
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    return p, A


def test_partition_covers_grid_once():
    w = workloads.configs.metasurface_sheet(interior=256, pml=20, parts=4, n_pillars=8, slot=32,
                                            substrate_rows=64, source_row=32)
    subs = ddm.partition(w.params())
    own = np.zeros((w.ny, w.nx), int)
    for s in subs:
        own[s.iy[0]:s.iy[1], s.ix[0]:s.ix[1]] += 1
        e = 24
        assert s.ox[0] == (s.ix[0] - e if s.kx > 0 else 0)
        assert s.oy[1] == (s.iy[1] + e if s.ky < 3 else w.ny)
    assert np.all(own == 1)
    # Interior blocks of 64 cells; the edge blocks carry the 20-cell PML.
    assert [s.ix for s in subs[:4]] == [(0, 84), (84, 148), (148, 212), (212, 296)]


def test_config_local_shapes():
    """The 8x8 split of a 1024 interior with a 20-cell PML gives local sides
    of 172 (edge) and 176 (interior); the 2x2 split of the 100 interior with a
    16-cell PML gives 90."""
    p = workloads.configs.metasurface_sheet.__defaults__  # noqa: F841 (documentation)
    params = dict(nx=1064, ny=1064, pml=(20,) * 4, px=8, py=8, overlap=8, local_pml=16)
    sides = sorted({s.ox[1] - s.ox[0] for s in ddm.partition(params)})
    assert sides == [172, 176]
    params = dict(nx=132, ny=132, pml=(16,) * 4, px=2, py=2, overlap=8, local_pml=16)
    assert {s.ox[1] - s.ox[0] for s in ddm.partition(params)} == {90}


def test_local_stretch_follows_global_away_from_local_pml():
    w = workloads.configs.small_random(nx=60, ny=50, pml=6, px=3, py=2, overlap=3, local_pml=5)
    p = w.params()
    sx, sxh, sy, syh = fdfd.global_axes(p)
    for s in ddm.partition(p):
        ls, lsh = ddm.local_axis(sx, sxh, s.ox, s.ix, s.ox[0] < s.ix[0], s.ox[1] > s.ix[1],
                                 3, 5, 3, 1e-8, p["k0"], 1.0)
        a = s.ox[0]
        # I_k plus the physical overlap keep the global values exactly.
        lo = s.ix[0] - (3 if s.ox[0] < s.ix[0] else 0)
        hi = s.ix[1] + (3 if s.ox[1] > s.ix[1] else 0)
        assert np.array_equal(ls[lo - a:hi - a], sx[lo:hi])
        assert np.array_equal(lsh[lo - a:hi - a + 1], sxh[lo:hi + 1])
        # The local PML has the same profile as a global PML of the same depth.
        if s.ox[1] > s.ix[1]:
            gs, gsh = fdfd.axis_stretch(5 + 5, 0, 5, 3, 1e-8, p["k0"], 1.0)
            assert np.allclose(ls[-5:], gs[-5:]) and np.allclose(lsh[-6:], gsh[-6:])


def test_single_subdomain_round_is_exact_inverse():
    """N = 1: Omega_1 is the whole grid, so one round is A^{-1} b."""
    w = workloads.configs.small_random(nx=40, ny=36, pml=6, px=1, py=1)
    p, A = _setup(w)
    B = ddm.SourceTransfer(p, w.eps_cells)
    b = w.b[0].ravel()
    assert fdfd.relres(A, B.apply(b), b) < 1e-13


@pytest.mark.parametrize("px,py", [(2, 2), (3, 2)])
def test_residual_vanishes_away_from_transfer_bands(px, py):
    """After the initial local solves (Eq. (14)) summed by Eq. (21), the global
    residual on I_k is exactly the source transferred from neighbours, so it is
    zero at every node whose stencil does not touch a neighbour's Omega_i."""
    w = workloads.configs.small_random(nx=70, ny=64, pml=6, px=px, py=py, overlap=3, local_pml=6)
    p, A = _setup(w)
    B = ddm.SourceTransfer(p, w.eps_cells)
    b = w.b[0].ravel()
    r = (b - A @ B.apply(b)).reshape(w.ny, w.nx)
    touched = np.zeros((w.ny, w.nx), bool)
    for s in B.subs:
        cover = np.zeros((w.ny, w.nx), bool)
        cover[s.oy[0]:s.oy[1], s.ox[0]:s.ox[1]] = True
        grow = cover.copy()
        grow[1:, :] |= cover[:-1, :]; grow[:-1, :] |= cover[1:, :]
        grow[:, 1:] |= cover[:, :-1]; grow[:, :-1] |= cover[:, 1:]
        own = np.zeros_like(cover)
        own[s.iy[0]:s.iy[1], s.ix[0]:s.ix[1]] = True
        # Nodes outside I_s whose stencil meets Omega_s receive s's field.
        touched |= grow & ~own
    scale = np.abs(b).max()
    assert np.abs(r[~touched]).max() < 1e-12 * scale
    assert np.abs(r[touched]).max() > 1e-6 * scale


def test_stationary_algorithm1_converges_to_direct():
    """Algorithm 1 (Jacobi rounds) converges to the full-domain solution (Fig. 5b)."""
    w = workloads.configs.cylinder_tfsf()
    p, A = _setup(w)
    B = ddm.SourceTransfer(p, w.eps_cells)
    b = w.b[0].ravel()
    x, hist = ddm.stationary(A, B, b, 14)
    assert hist[-1] < 1e-13
    assert all(h1 < h0 for h0, h1 in zip(hist[:8], hist[1:9]))
    xd = fdfd.solve_direct(A, b)
    assert fdfd.rel_l2(x, xd) < 1e-12


def test_fgmres_with_round_matches_direct():
    w = workloads.configs.cylinder_tfsf()
    p, A = _setup(w)
    B = ddm.SourceTransfer(p, w.eps_cells)
    b = w.b[0].ravel()
    x, info = krylov.fgmres(lambda v: A @ v, b, B.apply, tol=1e-12, restart=30)
    assert info["converged"] and info["iters"] <= 12
    assert fdfd.rel_l2(x, fdfd.solve_direct(A, b)) < 1e-11


def _ras_round(B, v, ny, nx):
    """Control for the pins below: the same local solves prolonged only on I_k
    (a restricted-additive reading the paper's Eq. (21) rules out)."""
    z = np.zeros((ny, nx), dtype=np.complex128)
    for s in B.subs:
        u = B.local_solve(s.k, B.restrict(v, s)).reshape(s.oy[1] - s.oy[0], s.ox[1] - s.ox[0])
        z[s.iy[0]:s.iy[1], s.ix[0]:s.ix[1]] += u[s.iy[0] - s.oy[0]:s.iy[1] - s.oy[0],
                                                 s.ix[0] - s.ox[0]:s.ix[1] - s.ox[0]]
    return z.ravel()


def _two_sub_vacuum(overlap=4, local_pml=10):
    w = workloads.configs.small_random(nx=120, ny=60, pml=10, px=2, py=1, overlap=overlap,
                                       local_pml=local_pml, seed=1)
    p = w.params()
    cells = np.ones_like(w.eps_cells)
    A = fdfd.global_matrix(p, cells)
    B = ddm.SourceTransfer(p, cells)
    b = np.zeros((w.ny, w.nx), dtype=np.complex128)
    b[w.ny // 2, 30] = 1.0                      # point source in I_1, far from the interface
    return w, A, B, b.ravel()


def test_round_residual_support_is_the_local_pml_band():
    """Eq. (21) sums the FULL local fields.  Where the local operator equals the
    global one (I_k and the `overlap` unstretched cells beyond it) the summed
    field satisfies the global equations, so after the initial solves the
    residual vanishes on the overlap cells next to the interface, including the
    first node across it, and lives only in the neighbour's local PML band
    (nodes c + o .. c + o + L).  A prolongation restricted to I_k leaves a
    residual right at the interface instead."""
    w, A, B, b = _two_sub_vacuum(overlap=4, local_pml=10)
    c = B.subs[1].ix[0]                          # first column of I_2
    o, L = w.overlap, w.local_pml
    col = np.abs((b - A @ B.apply(b)).reshape(w.ny, w.nx)).max(axis=0)
    assert col[c - o:c + o].max() < 1e-13        # both sides of the interface
    assert col[:c - o].max() < 1e-13 and col[c + o + L + 1:].max() < 1e-13
    band = col[c + o:c + o + L + 1]
    assert band.min() > 1e-6 and band.max() > 1e-3
    ras = np.abs((b - A @ _ras_round(B, b, w.ny, w.nx)).reshape(w.ny, w.nx)).max(axis=0)
    assert ras[c - 1:c + 1].min() > 1e-3         # the control fails the pin


def test_one_round_is_one_way_transfer_in_vacuum():
    """Two subdomains, vacuum, a point source in Omega_1: the initial solve
    (Eq. (14)) leaves the transferred source in Omega_2's band; one Jacobi round
    (Eqs. (18)-(21)) carries the wave on, so the residual drops to the level of
    the local PML's reflection (here ~7e-6 of |b| with 10 cubic cells, R = 1e-8),
    and a second round removes the reflections as well."""
    w, A, B, b = _two_sub_vacuum(overlap=4, local_pml=10)
    x, hist = ddm.stationary(A, B, b, 2)
    assert 1e-2 < hist[0] < 1.0
    assert hist[1] < 1e-4
    assert hist[2] < 1e-2 * hist[1]
    # the I_k-restricted control does not transfer the wave
    y = _ras_round(B, b, w.ny, w.nx)
    y = y + _ras_round(B, b - A @ y, w.ny, w.nx)
    assert fdfd.relres(A, y, b) > 0.1


# --- sweeping (multiplicative) orders -----------------------------------------

def test_sweep_stages_cover_every_subdomain():
    w = workloads.configs.small_random(nx=70, ny=64, pml=6, px=3, py=2, overlap=3, local_pml=6)
    subs = ddm.partition(w.params())
    for order in ddm.ORDERS:
        st = ddm.sweep_stages(subs, 3, 2, order)
        seen = sorted({k for stg in st for k in stg})
        assert seen == list(range(6))
        for stg in st:                  # no two subdomains of a stage are the same
            assert len(set(stg)) == len(stg)
    assert len(ddm.sweep_stages(subs, 3, 2, "rows")) == 3
    assert len(ddm.sweep_stages(subs, 3, 2, "rows_cols")) == 3 + 5
    assert len(ddm.sweep_stages(subs, 3, 2, "diagonal")) == 4 * 4 - 2
    # two colours, no two edge neighbours in one stage
    assert ddm.sweep_stages(subs, 3, 2, "checker") == [[0, 2, 4], [1, 3, 5]]
    for stg in ddm.sweep_stages(subs, 3, 2, "checker"):
        for a in stg:
            for b in stg:
                sa, sb = subs[a], subs[b]
                assert abs(sa.kx - sb.kx) + abs(sa.ky - sb.ky) != 1
    # additive = the Jacobi round
    B = ddm.SourceTransfer(w.params(), w.eps_cells)
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    v = w.b[0].ravel()
    assert np.allclose(ddm.sweep_apply(B, A, v, ddm.sweep_stages(subs, 3, 2, "additive")), B.apply(v),
                       rtol=0, atol=1e-13 * np.abs(B.apply(v)).max())


def test_one_column_sweep_carries_a_wave_through_both_subdomains():
    """Two subdomains side by side, vacuum, a point source in Omega_1: the
    staged order visits Omega_1 then Omega_2 (the second stage solves with the
    residual the first left, which is the transferred source), so ONE
    application reaches the local PML's reflection level, where the Jacobi
    round needs a second round (test_one_round_is_one_way_transfer_in_vacuum)."""
    w, A, B, b = _two_sub_vacuum(overlap=4, local_pml=10)
    stages = ddm.sweep_stages(B.subs, 2, 1, "rows_cols")      # [[0, 1], [0], [1], [0]]
    z1 = ddm.sweep_apply(B, A, b, [[0], [1]])
    assert fdfd.relres(A, z1, b) < 1e-4
    assert fdfd.relres(A, B.apply(b), b) > 1e-2
    # the full symmetric order only improves on that
    assert fdfd.relres(A, ddm.sweep_apply(B, A, b, stages), b) < 1e-4
    # the two-colour order of two subdomains is that one-way sweep
    assert ddm.sweep_stages(B.subs, 2, 1, "checker") == [[0], [1]]


@pytest.mark.parametrize("order", ["rows", "rows_cols", "diagonal", "checker"])
def test_fgmres_with_sweeps_matches_direct_in_fewer_iterations(order):
    """Any staged order is a fixed linear preconditioner: FGMRES converges to the
    direct solve, in fewer iterations than with the Jacobi round here."""
    w = workloads.configs.small_random(nx=96, ny=96, pml=8, px=3, py=3, overlap=3, local_pml=8,
                                       seed=12)
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    B = ddm.SourceTransfer(p, w.eps_cells)
    b = w.b[0].ravel()
    stages = ddm.sweep_stages(B.subs, 3, 3, order)
    x, info = krylov.fgmres(lambda v: A @ v, b, lambda v: ddm.sweep_apply(B, A, v, stages),
                            tol=1e-11, restart=40)
    _, add = krylov.fgmres(lambda v: A @ v, b, B.apply, tol=1e-11, restart=40)
    assert info["converged"] and fdfd.rel_l2(x, fdfd.solve_direct(A, b)) < 1e-9
    assert info["iters"] < add["iters"]


def test_single_subdomain_sweep_is_exact_inverse():
    w = workloads.configs.small_random(nx=40, ny=36, pml=6, px=1, py=1)
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    B = ddm.SourceTransfer(p, w.eps_cells)
    b = w.b[0].ravel()
    for order in ddm.ORDERS:
        z = ddm.sweep_apply(B, A, b, ddm.sweep_stages(B.subs, 1, 1, order))
        assert fdfd.relres(A, z, b) < 1e-13


def test_pooled_round_equals_the_round():
    """oracle.pool spreads the factors over worker processes; with complex128
    factors its round is SourceTransfer's (same arithmetic up to roundoff), with
    complex64 factors it is within single-precision rounding of it."""
    from oracle import pool
    w = workloads.configs.small_random(nx=70, ny=64, pml=6, px=3, py=2, overlap=3, local_pml=6)
    p = w.params()
    B = ddm.SourceTransfer(p, w.eps_cells)
    v = w.b[0].ravel()
    ref = B.apply(v)
    with pool.PooledSourceTransfer(p, w.eps_cells, 3) as P:
        assert np.linalg.norm(P.apply(v) - ref) < 1e-13 * np.linalg.norm(ref)
    with pool.PooledSourceTransfer(p, w.eps_cells, 2, np.complex64) as P:
        err = np.linalg.norm(P.apply(v) - ref) / np.linalg.norm(ref)
        assert 1e-9 < err < 1e-4


# --- the stop rule of Eq. (20) -------------------------------------------------

def test_overlap_energy_vanishes_without_overlap_and_in_one_way_transfer():
    """One subdomain has no overlapping region, so the energy of Eq. (20) is 0
    after the initial solve.  Two subdomains in vacuum with the source in
    Omega_1 (the setting of the paper's Fig. 4): the initial solve leaves an
    overlap field, and after one round the field in the overlapping regions is
    at the level of the local PML's reflection."""
    w = workloads.configs.small_random(nx=40, ny=36, pml=6, px=1, py=1)
    p = w.params()
    B1 = ddm.SourceTransfer(p, w.eps_cells)
    _, e = ddm.overlap_energy(B1, w.b[0].ravel())
    assert e == 0.0
    w2, A, B, b = _two_sub_vacuum(overlap=4, local_pml=10)
    x, en, hist = ddm.stationary_eq20(A, B, b, 1e-3, 3)
    assert en[0] > 0 and en[1] < 1e-3 * en[0]
    assert len(en) == 2 and hist[1] < 1e-4


def test_eq20_stop_rule_tracks_the_residual():
    """Run to the Eq. (20) threshold, the iterate is as close to the direct
    solve as the residual says (the energies fall with the residual)."""
    w = workloads.configs.cylinder_tfsf()
    p, A = _setup(w)
    B = ddm.SourceTransfer(p, w.eps_cells)
    b = w.b[0].ravel()
    x, en, hist = ddm.stationary_eq20(A, B, b, 1e-10, 30)
    assert en[-1] < 1e-10 * en[0]
    assert hist[-1] < 1e-9
    assert fdfd.rel_l2(x, fdfd.solve_direct(A, b)) < 1e-8
    # monotone decay over the first rounds, as the residual's
    assert all(e1 < e0 for e0, e1 in zip(en[:6], en[1:7]))
