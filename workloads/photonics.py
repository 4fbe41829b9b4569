"""Seeded silicon-photonics layouts on the FDFD grid (inputs only; no solver arithmetic).

A layout is a set of waveguide centre lines running left to right across the
physical region, each a function y(x): straight runs joined by raised-cosine
S-bends, y(x) = y0 + dy (1 - cos(pi (x - x0) / L)) / 2 on [x0, x0 + L], whose
largest curvature pi^2 |dy| / (2 L^2) is kept below 1 / r_min.  A Y-split is a
trunk whose two branches leave it with S-bends of opposite sign.  Cells are
filled by the fraction of their area inside a strip of the given width around
each centre line: the strip's vertical extent at a sub-column x is
|y - y(x)| < w / (2 cos theta) (theta the local slope angle, so that the width
across the guide is w), and a cell takes the mean over S sub-columns of the
exactly covered fraction of its height (the subcell rule of Eq. (8) with exact
integration along y).

The source is the fundamental guided mode of the cross-section at one column:
the eigenvector of the largest eigenvalue beta^2 of the tridiagonal operator
d^2/dy^2 + k0^2 eps(y) (three-point second difference, field zero beyond the
window), computed by SciPy's tridiagonal eigen-solver.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Path:
    """Centre line y(x) sampled as a piecewise function: list of segments
    (x0, x1, y0, dy) meaning y = y0 + dy (1 - cos(pi (x - x0) / (x1 - x0))) / 2
    on [x0, x1) (dy = 0: straight)."""
    segs: list = field(default_factory=list)

    def y(self, x):
        x = np.asarray(x, dtype=np.float64)
        out = np.full(x.shape, np.nan)
        for x0, x1, y0, dy in self.segs:
            m = (x >= x0) & (x < x1)
            if dy == 0.0:
                out[m] = y0
            else:
                out[m] = y0 + dy * (1.0 - np.cos(math.pi * (x[m] - x0) / (x1 - x0))) / 2.0
        return out

    def slope(self, x):
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape)
        for x0, x1, y0, dy in self.segs:
            if dy == 0.0:
                continue
            m = (x >= x0) & (x < x1)
            L = x1 - x0
            out[m] = dy * math.pi / (2.0 * L) * np.sin(math.pi * (x[m] - x0) / L)
        return out


def _bend_length(dy, r_min):
    """Shortest raised-cosine S-bend of offset dy with radius >= r_min."""
    return math.sqrt(math.pi ** 2 * abs(dy) * r_min / 2.0)


def route(x_start, x_end, y_start, y_lo, y_hi, r_min, rng, n_bends=3, max_dy=None):
    """A random route from (x_start, y_start) to x_end: straight runs joined by
    n_bends S-bends of random offsets keeping y in [y_lo, y_hi]."""
    p = Path()
    x, y = float(x_start), float(y_start)
    span = x_end - x_start
    max_dy = max_dy if max_dy is not None else 0.15 * (y_hi - y_lo)
    for _ in range(n_bends):
        run = rng.uniform(0.05, 0.2) * span
        dy = rng.uniform(-max_dy, max_dy)
        dy = min(max(dy, y_lo - y), y_hi - y)
        L = max(_bend_length(dy, r_min), 1.0)
        if x + run + L >= x_end:
            break
        p.segs.append((x, x + run, y, 0.0))
        x += run
        p.segs.append((x, x + L, y, dy))
        x += L
        y += dy
    p.segs.append((x, float(x_end) + 1.0, y, 0.0))
    return p


def y_split(trunk, x_split, half_dy, r_min, x_end):
    """Two branches leaving `trunk` at x_split with S-bends of +half_dy and
    -half_dy, then running straight to x_end (the trunk is cut at x_split)."""
    segs = [s for s in trunk.segs if s[0] < x_split]
    if segs:
        x0, x1, y0, dy = segs[-1]
        segs[-1] = (x0, min(x1, x_split), y0, dy)
    y_at = float(trunk.y(np.array([x_split - 1e-9]))[0])
    L = _bend_length(half_dy, r_min)
    branches = []
    for sgn in (1.0, -1.0):
        b = Path(list(segs))
        b.segs.append((x_split, x_split + L, y_at, sgn * half_dy))
        b.segs.append((x_split + L, float(x_end) + 1.0, y_at + sgn * half_dy, 0.0))
        branches.append(b)
    return branches


def strip_cells(nx, ny, paths, width, eps_core, eps_clad, subcols=16, dx=1.0, dy=1.0):
    """Cell permittivity map (ny+1, nx+1): the cladding plus, per cell, the mean
    over `subcols` sub-columns of the fraction of the cell's height inside the
    union of the strips (overlaps counted once by clipping at 1)."""
    cov = np.zeros((ny + 1, nx + 1))
    S = int(subcols)
    # sub-column centres of cell column c: x in [(c-1) dx, c dx]
    c = np.arange(nx + 1)
    xs = ((c[:, None] - 1) + (np.arange(S)[None, :] + 0.5) / S) * dx      # (nx+1, S)
    for path in paths:
        yc = path.y(xs.ravel()).reshape(xs.shape)
        ok = np.isfinite(yc)
        th = np.arctan(path.slope(xs.ravel()).reshape(xs.shape))
        half = 0.5 * width / np.cos(th)
        lo = np.where(ok, yc - half, np.inf) / dy
        hi = np.where(ok, yc + half, -np.inf) / dy
        # cell row d spans y in [(d-1), d] (units of dy)
        dmin = int(max(0, np.floor(np.nanmin(np.where(ok, lo, np.nan))) ))
        dmax = int(min(ny, np.ceil(np.nanmax(np.where(ok, hi, np.nan))) + 1))
        for d in range(dmin, dmax + 1):
            f = np.clip(np.minimum(hi, d) - np.maximum(lo, d - 1), 0.0, 1.0)   # (nx+1, S)
            cov[d] += f.mean(axis=1)
    cov = np.clip(cov, 0.0, 1.0)
    return (eps_clad + (eps_core - eps_clad) * cov).astype(np.complex128)


def strip_nodes(nx, ny, paths, width, eps_core, eps_clad, dx=1.0, dy=1.0):
    """Permittivity sampled at the nodes (i dx, j dy): core inside any strip."""
    out = np.full((ny, nx), complex(eps_clad), dtype=np.complex128)
    X = np.arange(nx) * dx
    Y = np.arange(ny)[:, None] * dy
    for path in paths:
        yc = path.y(X)
        th = np.arctan(path.slope(X))
        half = 0.5 * width / np.cos(th)
        inside = np.isfinite(yc)[None, :] & (np.abs(Y - yc[None, :]) < half[None, :])
        out[inside] = eps_core
    return out


def fundamental_mode(eps_column, k0, dy=1.0):
    """(beta^2, phi): the largest eigenpair of the tridiagonal d^2/dy^2 + k0^2 eps
    on the given column (real part of eps), phi normalised to unit 2-norm with a
    positive maximum."""
    from scipy.linalg import eigh_tridiagonal
    e = np.real(np.asarray(eps_column))
    n = e.size
    d = -2.0 / dy ** 2 + k0 ** 2 * e
    off = np.full(n - 1, 1.0 / dy ** 2)
    w, v = eigh_tridiagonal(d, off, select="i", select_range=(n - 1, n - 1))
    phi = v[:, 0]
    phi = phi / np.linalg.norm(phi)
    if phi[np.argmax(np.abs(phi))] < 0:
        phi = -phi
    return float(w[0]), phi
