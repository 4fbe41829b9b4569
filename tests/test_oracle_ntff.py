"""Pins of the near-to-far-field transform and the radar cross section
(oracle/ntff.py; the paper's Fig. 5a validation quantity)."""
import math

import numpy as np
import pytest
from scipy import special

import workloads
from oracle import fdfd, mie, ntff


def test_line_source_far_field_is_the_hankel_asymptote():
    """u = H0^(2)(k |r - r0|) sampled on the grid: F(phi) must equal
    -4j exp(j k rhat . r0) (the far field of the representation), to second
    order in h; the scattering width is 4 / k."""
    k = 2 * math.pi
    phis = np.linspace(0, 2 * math.pi, 16, endpoint=False)
    errs = []
    for ppw in (20, 40, 80):
        h = 1.0 / ppw
        n = int(round(3 / h))
        X, Y = np.meshgrid(np.arange(n) * h, np.arange(n) * h)
        r0 = (1.4, 1.6)
        u = special.hankel2(0, k * np.hypot(X - r0[0], Y - r0[1]))
        box = (int(0.5 / h), int(2.5 / h), int(0.5 / h), int(2.5 / h))
        F = ntff.far_field(u, h, h, box, k, phis)
        ex = -4j * np.exp(1j * k * (np.cos(phis) * r0[0] + np.sin(phis) * r0[1]))
        errs.append(np.abs(F - ex).max() / 4.0)
        assert np.allclose(ntff.rcs(u, h, h, box, k, phis), 4.0 / k, rtol=4 * errs[-1])
    assert errs[0] < 0.02 and errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5


def test_vacuum_scatters_nothing():
    phis = np.linspace(0, 2 * math.pi, 8, endpoint=False)
    assert np.abs(mie.coefficients(2.0, 0.7, 1.0)[1]).max() < 1e-15
    assert ntff.mie_rcs(2.0, 0.7, 1.0, phis).max() < 1e-28
    u = np.zeros((40, 40), dtype=np.complex128)
    assert ntff.rcs(u, 0.1, 0.1, (5, 30, 5, 30), 2.0, phis).max() == 0.0


def _cylinder_rcs_error(ppw, a=0.5, eps=4.0, half=1.25):
    h = 1.0 / ppw
    L = int(0.8 * ppw)
    n = int(round(2 * half / h)) + 2 * L
    c = (n - 1) / 2.0
    k0 = 2 * math.pi
    cells = workloads.geometry.cylinder(n, n, c * h, c * h, a, eps, dx=h, dy=h, subcells=16)
    p = dict(nx=n, ny=n, dx=h, dy=h, k0=k0, pml=(L,) * 4, pml_order=3, pml_R=1e-8)
    A = fdfd.global_matrix(p, cells)
    X, Y = np.meshgrid(np.arange(n) * h - c * h, np.arange(n) * h - c * h)
    einc = np.exp(-1j * k0 * (X + c * h))                  # unit plane wave along +x
    b = (-k0 ** 2 * (fdfd.node_eps(cells) - 1) * einc).ravel()
    u = fdfd.solve_direct(A, b).reshape(n, n)
    m = L + int(0.1 / h)                                   # contour 0.1 lambda inside the PML edge
    box = (m, n - 1 - m, m, n - 1 - m)
    phis = np.linspace(0, 2 * math.pi, 72, endpoint=False)
    s = ntff.rcs(u, h, h, box, k0, phis)
    ref = ntff.mie_rcs(k0, a, eps, phis)
    return np.linalg.norm(s - ref) / np.linalg.norm(ref)


@pytest.mark.slow
def test_fdfd_cylinder_rcs_matches_mie():
    """The RCS of the scattered-field FDFD solution of a dielectric cylinder
    (r = lambda/2, eps 4) against the Mie series.  sigma is quadratic in the
    field, so its relative error is about twice the field's (12% / 2.8% / 0.7%
    at 20 / 40 / 80 points per wavelength, test_oracle_mie.py) and falls at
    second order in h (the paper reports 3.68% for its own cylinder at 40)."""
    e = [_cylinder_rcs_error(ppw) for ppw in (20, 40, 80)]
    assert e[0] < 0.35 and e[1] < 0.09 and e[2] < 0.025, e
    assert e[1] < e[0] / 3.2 and e[2] < e[1] / 3.2, e
