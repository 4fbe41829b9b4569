"""Right-hand sides (sources) on the node grid; arrays are (ny, nx) complex128, x fastest.

These are inputs to the solve.  The paper supplies b in Eq. (4) (and the
scattered-field form in Eq. (7)); the physical prefactor j*omega*mu0 of
Eq. (14) does not change the discrete problem and is left to the caller.
"""
from __future__ import annotations

import math

import numpy as np


def discrete_wavenumber(k0, dx):
    """Wavenumber whose plane wave exp(-j kt x) satisfies the vacuum 3-point
    second difference exactly: (2/dx) asin(k0 dx / 2)."""
    return 2.0 / dx * math.asin(k0 * dx / 2.0)


def tfsf_plane_wave_x(nx, ny, dx, k0, col):
    """Total-field/scattered-field line source for a unit plane wave moving +x.

    The total-field region is every node column i >= col (which must lie in
    the unstretched interior, so the x-coupling across the line is 1/dx^2).
    With Q the indicator of that region and e_inc the discrete plane wave
    exp(-j kt x_i), the source is b = (A Q - Q A) e_inc; only the two columns
    next to the line are coupled by A across it, giving
        b[:, col-1] = +e_inc(x_col) / dx^2,   b[:, col] = -e_inc(x_{col-1}) / dx^2.
    """
    if not (1 <= col < nx):
        raise ValueError("TF/SF column out of range")
    kt = discrete_wavenumber(k0, dx)
    b = np.zeros((ny, nx), dtype=np.complex128)
    b[:, col - 1] = np.exp(-1j * kt * col * dx) / dx ** 2
    b[:, col] = -np.exp(-1j * kt * (col - 1) * dx) / dx ** 2
    return b


def plane_wave_x(nx, ny, dx, k0, col):
    """Discrete incident plane wave restricted to the total-field region (i >= col)."""
    kt = discrete_wavenumber(k0, dx)
    e = np.zeros((ny, nx), dtype=np.complex128)
    e[:, col:] = np.exp(-1j * kt * np.arange(col, nx) * dx)[None, :]
    return e


def point_dipole(nx, ny, i, j, amp=1.0):
    b = np.zeros((ny, nx), dtype=np.complex128)
    b[j, i] = amp
    return b


def current_sheet(nx, ny, row, amp=1.0):
    """b = amp on every node of one row (a line current; radiates plane waves up and down)."""
    b = np.zeros((ny, nx), dtype=np.complex128)
    b[row, :] = amp
    return b


def random_field(nx, ny, seed):
    """Seeded complex field with independent standard-normal real and imaginary parts."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))).astype(np.complex128)


def scattered_plane_wave(contrast, k0, theta, dx=1.0, dy=1.0):
    """Scattered-field source of a unit plane wave exp(-j k0 (x cos t + y sin t))
    (the form of Eq. (7)): b = -k0^2 (eps - 1) e_inc, with the permittivity
    contrast (eps - 1) given per node (ny, nx); the solution is the field
    scattered by the contrast."""
    ny, nx = contrast.shape
    X = np.arange(nx)[None, :] * dx
    Y = np.arange(ny)[:, None] * dy
    e_inc = np.exp(-1j * k0 * (X * math.cos(theta) + Y * math.sin(theta)))
    return (-(k0 ** 2) * contrast * e_inc).astype(np.complex128)
