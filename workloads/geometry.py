"""Seeded permittivity maps on the FDFD cell grid (inputs only; no solver arithmetic).

Grid convention shared by every consumer of these maps: nodes (i, j) with
0 <= i < nx, 0 <= j < ny sit at x = i*dx, y = j*dy.  The cell map has shape
(ny+1, nx+1); cell (c, d) is the dual cell whose corners are nodes
(c-1..c, d-1..d), i.e. it spans x in [(c-1)dx, c dx], y in [(d-1)dy, d dy].

Cell permittivities follow the subcell rule of the paper (Sec. 2.1, Eq. (8)):
each cell is split into S x S subcells, a subcell takes the permittivity of the
medium that contains its centre, and the cell value is the mean over its
subcells.  Shapes are painted in list order; a later shape wins where shapes
overlap.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Circle:
    cx: float
    cy: float
    r: float
    eps: complex

    def bbox(self):
        return self.cx - self.r, self.cx + self.r, self.cy - self.r, self.cy + self.r

    def inside(self, x, y):
        return (x - self.cx) ** 2 + (y - self.cy) ** 2 < self.r ** 2


@dataclass(frozen=True)
class Rect:
    x0: float
    x1: float
    y0: float
    y1: float
    eps: complex

    def bbox(self):
        return self.x0, self.x1, self.y0, self.y1

    def inside(self, x, y):
        return (x >= self.x0) & (x < self.x1) & (y >= self.y0) & (y < self.y1)


def subcell_raster(nx, ny, shapes, eps_bg=1.0, dx=1.0, dy=1.0, subcells=16, strip=8):
    """Cell permittivity map (ny+1, nx+1) complex128 by centre-in-shape subcell averaging.

    Painting is exact per subcell: strips of `strip` cell rows are expanded to
    their S x S subcells, every shape overlapping the strip overwrites the
    subcells whose centres it contains (in list order), and each cell takes the
    mean of its subcells.
    """
    S = int(subcells)
    cells = np.full((ny + 1, nx + 1), complex(eps_bg), dtype=np.complex128)
    off = (np.arange(S) + 0.5) / S
    boxes = [shp.bbox() for shp in shapes]
    for d0 in range(0, ny + 1, strip):
        d1 = min(ny + 1, d0 + strip)                 # cells d0..d1-1
        ylo, yhi = (d0 - 1) * dy, (d1 - 1) * dy      # strip extent
        act = [k for k, b in enumerate(boxes) if b[3] >= ylo and b[2] <= yhi]
        if not act:
            continue
        c0 = max(0, min(int(math.floor(boxes[k][0] / dx)) for k in act))
        c1 = min(nx, max(int(math.ceil(boxes[k][1] / dx)) + 1 for k in act))
        if c0 > c1:
            continue
        cs = np.arange(c0, c1 + 1)
        ds = np.arange(d0, d1)
        xs = ((cs[:, None] - 1 + off[None, :]) * dx).reshape(-1)
        ys = ((ds[:, None] - 1 + off[None, :]) * dy).reshape(-1)
        sub = np.full((len(ys), len(xs)), complex(eps_bg), dtype=np.complex128)
        for k in act:
            bx0, bx1, by0, by1 = boxes[k]
            ia = int(np.searchsorted(xs, bx0, side="left"))
            ib = int(np.searchsorted(xs, bx1, side="right"))
            ja = int(np.searchsorted(ys, by0, side="left"))
            jb = int(np.searchsorted(ys, by1, side="right"))
            if ia >= ib or ja >= jb:
                continue
            X, Y = np.meshgrid(xs[ia:ib], ys[ja:jb])
            hit = shapes[k].inside(X, Y)
            blk = sub[ja:jb, ia:ib]
            blk[hit] = shapes[k].eps
        cells[d0:d1, c0:c1 + 1] = sub.reshape(len(ds), S, len(cs), S).mean(axis=(1, 3))
    return cells


def cylinder(nx, ny, cx, cy, radius, eps_cyl, eps_bg=1.0, dx=1.0, dy=1.0, subcells=16):
    """One dielectric cylinder (circle) in a uniform background."""
    return subcell_raster(nx, ny, [Circle(cx, cy, radius, eps_cyl)], eps_bg, dx, dy, subcells)


def metasurface(nx, ny, pml, lam_cells, n_pillars, slot, substrate_rows, eps_pillar, eps_sub,
                seed, wmin=0.1, wmax=0.4, subcells=16):
    """Random metasurface: a half-plane substrate and rectangular pillars standing on it.

    The substrate fills every node row below `pml + substrate_rows` (extending
    into the lower PML, as a half-plane does).  Pillar k is centred in the
    slot [pml + k*slot, pml + (k+1)*slot) along x; its width and height are
    drawn uniformly in [wmin, wmax]*lambda from numpy's PCG64 with `seed`.
    """
    rng = np.random.default_rng(seed)
    ysub = pml + substrate_rows - 0.5
    shapes = [Rect(-1.0, nx + 1.0, -1.0, ysub, eps_sub)]
    for k in range(n_pillars):
        w = rng.uniform(wmin, wmax) * lam_cells
        h = rng.uniform(wmin, wmax) * lam_cells
        xc = pml + (k + 0.5) * slot - 0.5
        shapes.append(Rect(xc - w / 2, xc + w / 2, ysub, ysub + h, eps_pillar))
    return subcell_raster(nx, ny, shapes, 1.0, 1.0, 1.0, subcells)


def random_disk_shapes(nx, ny, pml, lam_cells, fill, nmin, nmax, rmin, rmax, rng):
    """Random dielectric disks (refractive index U(nmin, nmax), radius
    U(rmin, rmax)*lambda, uniform centres inside the physical region) drawn from
    `rng` until the summed disk area reaches `fill` of the physical area."""
    w = nx - 2 * pml
    h = ny - 2 * pml
    target = fill * w * h
    area = 0.0
    shapes = []
    while area < target:
        n = rng.uniform(nmin, nmax)
        r = rng.uniform(rmin, rmax) * lam_cells
        cx = pml + rng.uniform(0, w - 1)
        cy = pml + rng.uniform(0, h - 1)
        shapes.append(Circle(cx, cy, r, n * n))
        area += math.pi * r * r
    return shapes


def random_disks(nx, ny, pml, lam_cells, fill, nmin, nmax, rmin, rmax, seed, subcells=8):
    """Vacuum plus random dielectric disks (random_disk_shapes with a PCG64 of
    `seed`) rasterised on the cell grid."""
    shapes = random_disk_shapes(nx, ny, pml, lam_cells, fill, nmin, nmax, rmin, rmax,
                                np.random.default_rng(seed))
    return subcell_raster(nx, ny, shapes, 1.0, 1.0, 1.0, subcells)


def node_samples(nx, ny, shapes, eps_bg=1.0, dx=1.0, dy=1.0):
    """Permittivity sampled at the node positions (i dx, j dy): the medium that
    contains the node itself (later shapes win).  Used to shape sources, not
    the operator."""
    out = np.full((ny, nx), complex(eps_bg), dtype=np.complex128)
    for shp in shapes:
        x0, x1, y0, y1 = shp.bbox()
        i0, i1 = max(0, int(math.floor(x0 / dx))), min(nx, int(math.ceil(x1 / dx)) + 1)
        j0, j1 = max(0, int(math.floor(y0 / dy))), min(ny, int(math.ceil(y1 / dy)) + 1)
        if i0 >= i1 or j0 >= j1:
            continue
        X, Y = np.meshgrid(np.arange(i0, i1) * dx, np.arange(j0, j1) * dy)
        blk = out[j0:j1, i0:i1]
        blk[shp.inside(X, Y)] = shp.eps
    return out
