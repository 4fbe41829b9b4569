"""Pins for the Mie series and for the discretisation against it (Sec. 3.1).
CPU only."""
import math

import numpy as np
import pytest
from scipy import special

import workloads
from oracle import fdfd, mie


def test_jacobi_anger_convention():
    """The series convention: sum_n j^-n J_n(k r) e^{j n phi} = exp(-j k r cos phi)."""
    k, r = 2.3, np.linspace(0.1, 3.0, 7)
    phi = np.linspace(-3, 3, 11)
    R, P = np.meshgrid(r, phi)
    n = np.arange(-60, 61)
    s = sum((1j) ** (-nn) * special.jv(nn, k * R) * np.exp(1j * nn * P) for nn in n)
    assert np.abs(s - np.exp(-1j * k * R * np.cos(P))).max() < 1e-13


def test_vacuum_cylinder_scatters_nothing():
    x = np.linspace(-2, 2, 9)
    X, Y = np.meshgrid(x, x)
    assert np.abs(mie.scattered_field(2.0, 0.7, 1.0, X, Y)).max() < 1e-13


def test_boundary_continuity():
    """Total field and its radial derivative are continuous across r = a."""
    k0, a, eps = 2 * math.pi, 0.5, 4.0
    phi = np.linspace(-3.1, 3.1, 13)
    d = 1e-6
    def total(r):
        x, y = r * np.cos(phi), r * np.sin(phi)
        return mie.scattered_field(k0, a, eps, x, y) + np.exp(-1j * k0 * x)
    ein, eout = total(a - d), total(a + d)
    assert np.abs(ein - eout).max() < 1e-4
    din = (total(a - d) - total(a - 3 * d)) / (2 * d)
    dout = (total(a + 3 * d) - total(a + d)) / (2 * d)
    assert np.abs(din - dout).max() < 1e-3 * np.abs(din).max()


def test_series_converged():
    k0, a, eps = 2 * math.pi, 0.5, 4.0
    x = np.array([0.2, 0.9, -1.1]); y = np.array([0.1, -0.4, 0.7])
    n, an, bn, k1 = mie.coefficients(k0, a, eps)
    f1 = mie.scattered_field(k0, a, eps, x, y)
    f2 = mie.scattered_field(k0, a, eps, x, y, nmax=2 * n.max())
    assert np.abs(f1 - f2).max() < 1e-13


def _fdfd_vs_mie(ppw, half=1.25, a=0.5, eps=4.0):
    h = 1.0 / ppw
    L = int(0.8 * ppw)
    n = int(round(2 * half / h)) + 2 * L
    c = (n - 1) / 2.0
    k0 = 2 * math.pi
    cells = workloads.geometry.cylinder(n, n, c * h, c * h, a, eps, dx=h, dy=h, subcells=16)
    p = dict(nx=n, ny=n, dx=h, dy=h, k0=k0, pml=(L,) * 4, pml_order=3, pml_R=1e-8)
    A = fdfd.global_matrix(p, cells)
    X, Y = np.meshgrid(np.arange(n) * h - c * h, np.arange(n) * h - c * h)
    einc = np.exp(-1j * k0 * (X + c * h))
    b = (-k0 ** 2 * (fdfd.node_eps(cells) - 1) * einc).ravel()     # scattered-field source, Eq. (7)
    x = fdfd.solve_direct(A, b).reshape(n, n)
    ref = mie.scattered_field(k0, a, eps, X, Y) * np.exp(-1j * k0 * c * h)
    mask = np.zeros((n, n), bool)
    mask[L:n - L, L:n - L] = True
    mask &= np.abs(np.hypot(X, Y) - a) >= 2 * h
    return np.linalg.norm((x - ref)[mask]) / np.linalg.norm(ref[mask])


@pytest.mark.slow
def test_fdfd_converges_to_mie_second_order():
    """Scattered-field FDFD (Eq. (7) with the PML of Eq. (9)) converges to the
    Mie series at second order in h (five-point stencil, subcell averaging)."""
    errs = {ppw: _fdfd_vs_mie(ppw) for ppw in (20, 40, 80)}
    o1 = math.log2(errs[20] / errs[40])
    o2 = math.log2(errs[40] / errs[80])
    assert o1 > 1.8 and o2 > 1.8, errs
    assert errs[80] < 1e-2, errs
