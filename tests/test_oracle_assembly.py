"""Pins for the oracle's assembly (Eqs. (2), (3), (9)-(13)) against closed forms,
invariants and brute force.  CPU only."""
import math

import numpy as np
import pytest

import workloads
from oracle import fdfd


def _params(nx, ny, k0, pml=(0, 0, 0, 0), m=3, R=1e-8, dx=1.0, dy=1.0):
    return dict(nx=nx, ny=ny, dx=dx, dy=dy, k0=k0, pml=pml, pml_order=m, pml_R=R)


@pytest.mark.parametrize("nx,ny,dx,dy", [(9, 7, 1.0, 1.0), (12, 5, 0.7, 1.3)])
def test_interior_stencil_closed_form_eigenpairs(nx, ny, dx, dy):
    """No PML, uniform medium, Dirichlet box: the discrete sine modes are
    eigenvectors with eigenvalue -(4/dx^2) sin^2(pi p/(2(nx+1)))
    - (4/dy^2) sin^2(pi q/(2(ny+1))) + k0^2 eps."""
    k0, eps = 0.9, 2.5 - 0.1j
    cells = np.full((ny + 1, nx + 1), eps, dtype=complex)
    A = fdfd.global_matrix(_params(nx, ny, k0, dx=dx, dy=dy), cells)
    i = np.arange(nx)
    j = np.arange(ny)
    for p in range(1, nx + 1):
        for q in (1, 2, ny):
            v = np.outer(np.sin(math.pi * q * (j + 1) / (ny + 1)), np.sin(math.pi * p * (i + 1) / (nx + 1))).ravel()
            lam = (-(4 / dx ** 2) * math.sin(math.pi * p / (2 * (nx + 1))) ** 2
                   - (4 / dy ** 2) * math.sin(math.pi * q / (2 * (ny + 1))) ** 2 + k0 ** 2 * eps)
            assert np.linalg.norm(A @ v - lam * v) <= 1e-12 * np.linalg.norm(v) * abs(lam)


def test_node_eps_is_four_cell_mean():
    """Eq. (3) on a map with one non-unit cell: that cell touches exactly its
    four corner nodes, each with weight 1/4."""
    cells = np.ones((6, 7), dtype=complex)
    cells[3, 4] = 9.0
    eb = fdfd.node_eps(cells)
    assert eb.shape == (5, 6)
    hot = np.argwhere(np.abs(eb - 1) > 1e-15)
    assert sorted(map(tuple, hot)) == [(2, 3), (2, 4), (3, 3), (3, 4)]
    assert np.allclose(eb[2:4, 3:5], 3.0)


def test_reciprocity_with_pml():
    """S = diag(s_x s_y) A is complex symmetric, so Green's functions between
    physical-interior nodes are reciprocal, G(a, b) = G(b, a), whatever the
    medium.  An assembly whose coupling i -> i+1 and i+1 -> i use different
    half-point stretches breaks this."""
    w = workloads.configs.cylinder_tfsf(interior=40, pml=10, lam=10.0, parts=1)
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    n = w.nx
    rng = np.random.default_rng(7)
    pts = [(int(rng.integers(10, n - 10)), int(rng.integers(10, n - 10))) for _ in range(4)]
    G = np.zeros((4, 4), dtype=complex)
    for a, (ia, ja) in enumerate(pts):
        x = fdfd.solve_direct(A, workloads.sources.point_dipole(n, n, ia, ja).ravel())
        for bb, (ib, jb) in enumerate(pts):
            G[bb, a] = x[jb * n + ib]
    assert np.abs(G - G.T).max() <= 1e-12 * np.abs(G).max()
    # Also holds with a PML node as source/receiver once scaled by s_x s_y.
    sx, sxh, sy, syh = fdfd.global_axes(p)
    D = np.outer(sy, sx).ravel()
    S = (A.multiply(D[:, None])).tocsr()
    assert abs(S - S.T).max() <= 1e-12 * abs(S).max()


def test_dense_equals_superlu_with_pml():
    """Brute force: dense LAPACK and SuperLU agree on a tiny PML problem."""
    w = workloads.configs.small_random(nx=24, ny=20, pml=6, px=1, py=1)
    A = fdfd.global_matrix(w.params(), w.eps_cells)
    b = w.b[0].ravel()
    xd = fdfd.solve_dense(A, b)
    xs = fdfd.solve_direct(A, b)
    assert fdfd.rel_l2(xs, xd) <= 1e-12
    assert fdfd.relres(A, xd, b) <= 1e-13


def test_tfsf_source_matches_commutator():
    """The generator's TF/SF line equals (A Q - Q A) e_inc with the oracle's A."""
    w = workloads.configs.cylinder_tfsf(interior=40, pml=10, lam=10.0, parts=1)
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    col = w.meta["tfsf_col"]
    einc = workloads.sources.plane_wave_x(w.nx, w.ny, 1.0, p["k0"], 0).ravel()
    Q = np.zeros((w.ny, w.nx)); Q[:, col:] = 1
    Q = Q.ravel()
    ref = A @ (Q * einc) - Q * (A @ einc)
    assert np.abs(ref - w.b[0].ravel()).max() <= 1e-13


def test_tfsf_vacuum_leakage_small():
    """In vacuum the TF/SF line injects the plane wave into the total-field
    region and (nearly) nothing into the scattered-field region; the residue
    comes from the Dirichlet rows behind the y-PML."""
    w = workloads.configs.cylinder_tfsf(interior=60, pml=16, lam=20.0, parts=1, eps_cyl=1.0)
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    x = fdfd.solve_direct(A, w.b[0].ravel()).reshape(w.ny, w.nx)
    col, L = w.meta["tfsf_col"], 16
    inc = workloads.sources.plane_wave_x(w.nx, w.ny, 1.0, p["k0"], col)
    phys = (slice(L, w.ny - L), slice(L, w.nx - L))
    # Scattered-field side: leakage only; total-field side within 30 cells of
    # the line: the plane wave (the deviation grows towards the far x-PML
    # corners, where the wave meets the Dirichlet rows behind the y-PMLs).
    err_tf = np.abs(x - inc)[phys][:, col - L + 1:col - L + 30].max()
    err_sf = np.abs(x)[phys][:, :col - L - 1].max()
    assert err_tf < 1e-3 and err_sf < 1e-4


@pytest.mark.parametrize("dx,dy", [(1.0, 1.0), (0.6, 1.4)])
def test_line_flux_discrete_poynting_identity(dx, dy):
    """For any field E and a box of nodes, the sum over the box of
    Im(conj(E) * Laplacian_h E) dx dy (the five-point Laplacian, written here
    independently) equals -2 k0 times the net power flowing out through the
    four grid lines around the box (the discrete Poynting theorem; a dropped
    conjugate, a wrong sign or a transposed axis in line_flux fails it)."""
    nx, ny, k0 = 23, 17, 0.7
    rng = np.random.default_rng(5)
    E = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    x0, x1, y0, y1 = 4, 19, 3, 12
    s = 0.0
    for j in range(y0, y1):
        for i in range(x0, x1):
            lap = ((E[j, i + 1] - 2 * E[j, i] + E[j, i - 1]) / dx ** 2
                   + (E[j + 1, i] - 2 * E[j, i] + E[j - 1, i]) / dy ** 2)
            s += (np.conj(E[j, i]) * lap).imag * dx * dy
    f = lambda axis, index, lo, hi: fdfd.line_flux(E, nx, ny, axis, index, lo, hi, k0, dx, dy)
    out = (f(0, x1 - 1, y0, y1) - f(0, x0 - 1, y0, y1)
           + f(1, y1 - 1, x0, x1) - f(1, y0 - 1, x0, x1))
    assert abs(s + 2 * k0 * out) <= 1e-12 * abs(s)


@pytest.mark.parametrize("direction", [1, -1])
def test_line_flux_of_a_plane_wave(direction):
    """E = exp(-j beta y) (a wave towards +y for exp(+j w t)): the power through
    any horizontal line of width W is W sin(beta dy) / (2 k0 dy), which tends
    to W beta / (2 k0), the flux 1/2 |E|^2 / eta0 of a unit plane wave, as dy
    -> 0; towards -y it is the negative."""
    nx, ny, k0 = 12, 30, 0.5
    for dy in (1.0, 0.1, 0.01):
        beta = k0
        y = np.arange(ny) * dy
        E = np.tile(np.exp(-1j * direction * beta * y)[:, None], (1, nx))
        for j in (0, 7, ny - 2):
            u = fdfd.line_flux(E, nx, ny, 1, j, 2, 10, k0, 1.0, dy)
            assert u == pytest.approx(direction * 8 * math.sin(beta * dy) / (2 * k0 * dy), rel=1e-12)
    assert fdfd.line_flux(E, nx, ny, 1, 3, 2, 10, k0, 1.0, 0.01) == pytest.approx(direction * 8 / 2,
                                                                                rel=1e-4)
