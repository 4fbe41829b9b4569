"""FP64 CPU oracle: FDFD assembly with SC-PML and the global direct solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library.

Everything is plain NumPy/SciPy in complex128, written from the paper:
  * 2D TM wave equation, Eq. (1); five-point stencil, Eq. (2);
  * node permittivity as the mean of the four surrounding cells, Eq. (3);
  * linear system A e = b, Eq. (4);
  * stretched-coordinate PML operator, Eq. (9), with the stretch factor of
    Eq. (10), the polynomial grading of Eqs. (11)-(12) and sigma_max of Eq. (13).
Readings where the paper is silent or garbled:
  * time convention exp(+j w t): Eq. (10) and (13) taken literally give
    s = 1 - j|sigma|/(w eps0), which absorbs outgoing exp(-j k r) waves;
  * sigma/(w eps0) = (m+1)|ln R| / (2 k0 L dlt) * (rho / (L dlt))^m with the
    depth rho = (u - 1/2) dlt at integer PML node u and rho = u dlt at half node
    u (+1/2); eta*eps0*w = k0 turns Eq. (13) into this dimensionless form;
  * the field vanishes on the virtual nodes one step outside the grid
    (Dirichlet behind the PML).

Grid conventions: nodes (i, j), 0 <= i < nx, 0 <= j < ny, flat index j*nx + i
(x fastest).  Cell map shape (ny+1, nx+1); cell (c, d) has corner nodes
(c-1..c, d-1..d).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------
# PML stretch factors, Eqs. (10)-(13)
# ---------------------------------------------------------------------------

def sigma_hat_max(L, m, R, k0, dlt):
    """Peak normalised conductivity sigma_max/(w eps0) of Eq. (13).

    Eq. (13): sigma_max = (m+1) ln R / (2 eta d), d = L*dlt the PML depth,
    eta = 120 pi.  Dividing by w*eps0 and using eta*eps0*w = w/c = k0 gives
    (m+1) ln R / (2 k0 L dlt), negative for R < 1.
    """
    return (m + 1) * math.log(R) / (2.0 * k0 * L * dlt)


def stretch(depth, L, m, R, k0, dlt):
    """s = 1 + j sigma/(w eps0) at PML depth `depth` (Eq. (10)), with the
    polynomial grading (depth/(L dlt))^m of Eqs. (11)-(12)."""
    return 1.0 + 1j * sigma_hat_max(L, m, R, k0, dlt) * (depth / (L * dlt)) ** m


def axis_stretch(n, pml_lo, pml_hi, m, R, k0, dlt):
    """Stretch factors along one axis of the global grid.

    Returns (s, sh): s[i] at node i (0 <= i < n) and sh[i] at the half point
    i - 1/2 (0 <= i <= n).  A PML of L cells on the low side occupies nodes
    0..L-1; node L-u is PML node u (Eq. (11), depth (u-1/2) dlt) and the half
    point (L-u) - 1/2 is half node u (Eq. (12), depth u dlt), u = 0 being the
    interface (s = 1).  The high side mirrors this.
    """
    s = np.ones(n, dtype=np.complex128)
    sh = np.ones(n + 1, dtype=np.complex128)
    if pml_lo > 0:
        L = pml_lo
        for u in range(1, L + 1):
            s[L - u] = stretch((u - 0.5) * dlt, L, m, R, k0, dlt)
        for u in range(0, L + 1):
            sh[L - u] = stretch(u * dlt, L, m, R, k0, dlt)
    if pml_hi > 0:
        L = pml_hi
        for u in range(1, L + 1):
            s[n - L - 1 + u] = stretch((u - 0.5) * dlt, L, m, R, k0, dlt)
        for u in range(0, L + 1):
            sh[n - L + u] = stretch(u * dlt, L, m, R, k0, dlt)
    return s, sh


# ---------------------------------------------------------------------------
# Node permittivity, Eq. (3)
# ---------------------------------------------------------------------------

def node_eps(eps_cells):
    """Mean of the four cells that share node (i, j), Eq. (3)."""
    e = np.asarray(eps_cells, dtype=np.complex128)
    return 0.25 * (e[:-1, :-1] + e[:-1, 1:] + e[1:, :-1] + e[1:, 1:])


# ---------------------------------------------------------------------------
# Matrix, Eqs. (2) and (9)
# ---------------------------------------------------------------------------

def assemble(eps_cells, k0, dx, dy, sx, sxh, sy, syh):
    """Sparse A of Eq. (9) discretised by Eq. (2) on the node grid.

    Row (i, j):
      coefficient of E(i-1, j) = 1 / (dx^2 s_x[i] s_x[i-1/2]),
      coefficient of E(i+1, j) = 1 / (dx^2 s_x[i] s_x[i+1/2]),
      likewise in y with s_y,
      diagonal = k0^2 * eps_bar(i, j) - (sum of the four coefficients),
    where a neighbour outside the grid is a Dirichlet zero (its coefficient
    still enters the diagonal).  With s = 1 this is exactly Eq. (2).
    """
    eb = node_eps(eps_cells)
    ny, nx = eb.shape
    assert len(sx) == nx and len(sxh) == nx + 1 and len(sy) == ny and len(syh) == ny + 1
    rows, cols, vals = [], [], []
    idx = np.arange(nx * ny).reshape(ny, nx)
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    cw = 1.0 / (dx * dx * sx[I] * sxh[I])          # towards i-1 (half point i-1/2 = sxh[i])
    ce = 1.0 / (dx * dx * sx[I] * sxh[I + 1])      # towards i+1 (half point i+1/2 = sxh[i+1])
    cs = 1.0 / (dy * dy * sy[J] * syh[J])
    cn = 1.0 / (dy * dy * sy[J] * syh[J + 1])
    diag = k0 * k0 * eb - (cw + ce + cs + cn)
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(diag.ravel())
    m = I > 0
    rows.append(idx[m]); cols.append(idx[m] - 1); vals.append(cw[m])
    m = I < nx - 1
    rows.append(idx[m]); cols.append(idx[m] + 1); vals.append(ce[m])
    m = J > 0
    rows.append(idx[m]); cols.append(idx[m] - nx); vals.append(cs[m])
    m = J < ny - 1
    rows.append(idx[m]); cols.append(idx[m] + nx); vals.append(cn[m])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nx * ny, nx * ny))
    return A


def global_axes(p):
    """Global stretch arrays for a parameter dict (see workloads.configs.Workload.params)."""
    pxl, pxh, pyl, pyh = p["pml"]
    sx, sxh = axis_stretch(p["nx"], pxl, pxh, p["pml_order"], p["pml_R"], p["k0"], p["dx"])
    sy, syh = axis_stretch(p["ny"], pyl, pyh, p["pml_order"], p["pml_R"], p["k0"], p["dy"])
    return sx, sxh, sy, syh


def global_matrix(p, eps_cells):
    sx, sxh, sy, syh = global_axes(p)
    return assemble(eps_cells, p["k0"], p["dx"], p["dy"], sx, sxh, sy, syh)


# ---------------------------------------------------------------------------
# Direct solves (the plain definition of the result: A e = b, Eq. (4))
# ---------------------------------------------------------------------------

def solve_dense(A, b):
    """Brute force: dense LAPACK solve (tiny systems only)."""
    return np.linalg.solve(A.toarray(), b)


def solve_direct(A, b, refine=1):
    """SuperLU factorisation plus `refine` steps of iterative refinement."""
    lu = spla.splu(A.tocsc())
    x = lu.solve(b)
    for _ in range(refine):
        x = x + lu.solve(b - A @ x)
    return x


def relres(A, x, b):
    return np.linalg.norm(b - A @ x) / np.linalg.norm(b)


def rel_l2(x, xref):
    return np.linalg.norm(np.ravel(x) - np.ravel(xref)) / np.linalg.norm(np.ravel(xref))


def line_flux(E, nx, ny, axis, index, lo, hi, k0, dx, dy):
    """Time-averaged power per unit length through a grid line: the line
    integral U = 1/2 int_l Re(E x H*) of Sec. 3.2 for E = E_z z.  The line lies
    between node rows index and index + 1 (axis 1: constant y, nodes x in
    [lo, hi), power flowing towards +y) or node columns index and index + 1
    (axis 0: constant x, nodes y in [lo, hi), towards +x).  H from Faraday's law
    with exp(+j w t) and w mu = k0 (fields normalised so that eta0 = 1):
    H_x = (j / k0) dE_z/dy and H_y = -(j / k0) dE_z/dx, so the y component of
    the power flow is 1/2 Re(E_z conj(H_x)) and the x component
    -1/2 Re(E_z conj(H_y)); on the line E_z is the mean of the two node rows and
    the derivative their difference over the step.  Parity unpinned against the
    paper (it prints no worked value); pinned by the discrete Poynting identity
    and the discrete plane wave in tests/test_oracle_assembly.py."""
    F = np.asarray(E, dtype=np.complex128).reshape(ny, nx)
    if axis == 1:
        a, b, d, dl = F[index, lo:hi], F[index + 1, lo:hi], dy, dx
    else:
        a, b, d, dl = F[lo:hi, index], F[lo:hi, index + 1], dx, dy
    e_mid = 0.5 * (a + b)
    h = 1j / k0 * (b - a) / d              # H_x (axis 1) or -H_y (axis 0) on the line
    return 0.5 * float(np.sum(np.real(e_mid * np.conj(h)))) * dl
