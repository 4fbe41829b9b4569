"""FP64 CPU oracle: near-to-far-field transform and the 2D radar cross section.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper validates its cylinder result by the RCS against the Mie series
(Sec. 3.1, Fig. 5a).  Outside a closed contour C that encloses every source and
scatterer the scattered field u obeys (nabla^2 + k0^2) u = 0 with the
radiation condition, so Green's representation with the outgoing 2D Green's
function (j/4) H0^(2)(k0 |r - r'|) holds, and its large-argument form gives
    u(rho, phi) ~ (j/4) sqrt(2 / (pi k0 rho)) exp(-j (k0 rho - pi/4)) F(phi),
    F(phi) = int_C [du/dn' - j k0 (rhat . n') u] exp(j k0 rhat . r') dl'
(n' the outward normal, rhat = (cos phi, sin phi)), and the scattering width
    sigma(phi) = lim 2 pi rho |u|^2 / |E_inc|^2 = |F|^2 / (4 k0)
for a unit incident wave.  On the grid, C is the rectangle through the half-node
lines x = (i0 + 1/2) dx, (i1 + 1/2) dx, y = (j0 + 1/2) dy, (j1 + 1/2) dy; on
each edge u is the mean of the two node lines it separates and du/dn their
difference over the step (the line of stf_line_flux), integrated by the
midpoint rule over the nodes strictly inside the edge's span.

The Mie reference: with E_s = sum_n a_n j^-n H_n^(2)(k0 r) e^{j n phi} (oracle.mie),
sigma(phi) = (4 / k0) |sum_n a_n e^{j n phi}|^2.
"""
from __future__ import annotations

import numpy as np

from . import mie


def far_field(u, dx, dy, box, k0, phis):
    """F(phi) of the field u (ny, nx) on the contour box = (i0, i1, j0, j1)
    (node coordinates x = i dx, y = j dy)."""
    u = np.asarray(u).reshape(np.asarray(u).shape)
    i0, i1, j0, j1 = box
    phis = np.asarray(phis, dtype=float)
    c, s = np.cos(phis), np.sin(phis)
    F = np.zeros(phis.shape, dtype=np.complex128)
    xs = np.arange(i0 + 1, i1 + 1) * dx
    ys = np.arange(j0 + 1, j1 + 1) * dy
    for row, nrm in ((j0, -1.0), (j1, 1.0)):               # bottom, top edges
        a, b = u[row, i0 + 1:i1 + 1], u[row + 1, i0 + 1:i1 + 1]
        um, dn = 0.5 * (a + b), (b - a) / dy * nrm
        yl = (row + 0.5) * dy
        ph = np.exp(1j * k0 * (np.outer(c, xs) + s[:, None] * yl))
        F += ((dn[None, :] - 1j * k0 * (s * nrm)[:, None] * um[None, :]) * ph).sum(axis=1) * dx
    for col, nrm in ((i0, -1.0), (i1, 1.0)):               # left, right edges
        a, b = u[j0 + 1:j1 + 1, col], u[j0 + 1:j1 + 1, col + 1]
        um, dn = 0.5 * (a + b), (b - a) / dx * nrm
        xl = (col + 0.5) * dx
        ph = np.exp(1j * k0 * (c[:, None] * xl + np.outer(s, ys)))
        F += ((dn[None, :] - 1j * k0 * (c * nrm)[:, None] * um[None, :]) * ph).sum(axis=1) * dy
    return F


def rcs(u, dx, dy, box, k0, phis):
    """Scattering width sigma(phi) = |F|^2 / (4 k0) of the scattered field u."""
    return np.abs(far_field(u, dx, dy, box, k0, phis)) ** 2 / (4.0 * k0)


def mie_rcs(k0, a, eps, phis):
    """sigma(phi) of the dielectric cylinder from the Mie coefficients."""
    n, an, _, _ = mie.coefficients(k0, a, eps)
    phis = np.asarray(phis, dtype=float)
    s = (an[None, :] * np.exp(1j * np.outer(phis, n))).sum(axis=1)
    return 4.0 / k0 * np.abs(s) ** 2
