"""Workload descriptions with their seeded inputs.

All lengths are in grid cells (dx = dy = 1), so k0 = 2*pi/lambda_cells; only
k0*dx enters the discrete problem.  Each config returns a plain dict holding
the solver parameters and the input arrays (cell permittivity map and source).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import geometry, sources


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    k0: float
    pml: tuple            # global PML cells (x-, x+, y-, y+)
    pml_order: int
    pml_R: float
    px: int
    py: int
    overlap: int
    local_pml: int
    local_pml_order: int
    local_pml_R: float
    eps_cells: np.ndarray   # (ny+1, nx+1) complex128
    b: np.ndarray           # (nrhs, ny, nx) complex128
    dx: float = 1.0
    dy: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def ndof(self):
        return self.nx * self.ny

    def params(self, **over):
        d = dict(nx=self.nx, ny=self.ny, dx=self.dx, dy=self.dy, k0=self.k0, pml=tuple(self.pml),
                 pml_order=self.pml_order, pml_R=self.pml_R, px=self.px, py=self.py,
                 overlap=self.overlap, local_pml=self.local_pml,
                 local_pml_order=self.local_pml_order, local_pml_R=self.local_pml_R)
        d.update(over)
        return d


def cylinder_tfsf(interior=100, pml=16, lam=20.0, radius_lam=0.5, eps_cyl=4.0, parts=2,
                  overlap=8, local_pml=16, subcells=16):
    """Dielectric cylinder at the grid centre lit by a +x plane wave through a
    TF/SF line at interior column 2 (default: 100x100 interior, 16-cell PML,
    lambda = 20 cells, r = lambda/2, eps = 4, 2x2 subdomains, overlap 8)."""
    n = interior + 2 * pml
    c = (n - 1) / 2.0
    k0 = 2 * math.pi / lam
    cells = geometry.cylinder(n, n, c, c, radius_lam * lam, eps_cyl, subcells=subcells)
    col = pml + 2
    b = sources.tfsf_plane_wave_x(n, n, 1.0, k0, col)[None]
    return Workload("cylinder_tfsf_%d" % n, n, n, k0, (pml,) * 4, 3, 1e-8, parts, parts, overlap,
                    local_pml, 3, 1e-8, cells, b,
                    meta=dict(centre=(c, c), radius=radius_lam * lam, eps_cyl=eps_cyl, tfsf_col=col,
                              lam=lam))


def metasurface_sheet(interior=1024, pml=20, lam=30.0, parts=8, overlap=8, local_pml=16, seed=2,
                      n_pillars=None, slot=16, substrate_rows=256, source_row=128, subcells=16,
                      nrhs=1):
    """Random metasurface (pillars eps 12.25 on an eps 2.13 substrate) lit by a
    current sheet inside the substrate (default 1024x1024 interior, 20-cell PML,
    lambda = 30 cells, 8x8 subdomains, overlap 8, seed 2).  nrhs > 1 adds
    sheets at further substrate rows (source_row - 64, + 64, + 96, ...)."""
    n = interior + 2 * pml
    if n_pillars is None:
        n_pillars = interior // slot
    k0 = 2 * math.pi / lam
    cells = geometry.metasurface(n, n, pml, lam, n_pillars, slot, substrate_rows, 12.25, 2.13, seed,
                                 subcells=subcells)
    offs = [0, -64, 64, 96, -96, 32, -32, 112][:nrhs]
    if nrhs > len(offs) or any(not 0 < source_row + o < substrate_rows for o in offs):
        raise ValueError("sheet rows must lie inside the substrate")
    b = np.stack([sources.current_sheet(n, n, pml + source_row + o) for o in offs])
    return Workload("metasurface_%d" % n, n, n, k0, (pml,) * 4, 3, 1e-8, parts, parts, overlap,
                    local_pml, 3, 1e-8, cells, b, meta=dict(seed=seed, lam=lam))


def small_random(nx=48, ny=40, pml=6, lam=12.0, px=2, py=2, overlap=2, local_pml=6, seed=0,
                 nrhs=1):
    """Small random-medium problem for fast parity tests: smooth random
    permittivity in [1, 4] with a small loss, random complex sources."""
    rng = np.random.default_rng(seed)
    base = rng.uniform(1.0, 4.0, size=(ny + 1, nx + 1))
    cells = (base + 0.01j * rng.uniform(0, 1, size=base.shape)).astype(np.complex128)
    b = np.stack([sources.random_field(nx, ny, seed * 1000 + r + 1) for r in range(nrhs)])
    k0 = 2 * math.pi / lam
    return Workload("random_%dx%d" % (nx, ny), nx, ny, k0, (pml,) * 4, 3, 1e-8, px, py, overlap,
                    local_pml, 3, 1e-8, cells, b, meta=dict(seed=seed))


def disks_problem(k, sides=(256, 384, 512, 768), pml=16, block=128, overlap=8, local_pml=16,
                  nrhs=4, seed0=300, subcells=8):
    """Problem k of the batched workload: a square interior of side drawn from
    `sides` plus a 16-cell PML, vacuum with random dielectric disks (n in
    [1.4, 3.5], radius [0.15, 0.5] lambda, 30% area fill), lambda uniform in
    [16, 40] cells, side/128 subdomains per axis, and `nrhs` right-hand sides,
    each with probability 1/2 a plane wave at a random angle (scattered-field
    source) or a point dipole at a random interior node.  Seed seed0 + k."""
    rng = np.random.default_rng(seed0 + k)
    side = int(rng.choice(np.asarray(sides)))
    lam = float(rng.uniform(16.0, 40.0))
    n = side + 2 * pml
    k0 = 2 * math.pi / lam
    shapes = geometry.random_disk_shapes(n, n, pml, lam, 0.30, 1.4, 3.5, 0.15, 0.5, rng)
    cells = geometry.subcell_raster(n, n, shapes, 1.0, 1.0, 1.0, subcells)
    contrast = geometry.node_samples(n, n, shapes) - 1.0
    bs, kinds = [], []
    for _ in range(nrhs):
        if rng.uniform() < 0.5:
            th = float(rng.uniform(0.0, 2 * math.pi))
            bs.append(sources.scattered_plane_wave(contrast, k0, th))
            kinds.append(("plane", th))
        else:
            i, j = (int(v) for v in rng.integers(pml, pml + side, size=2))
            bs.append(sources.point_dipole(n, n, i, j))
            kinds.append(("dipole", (i, j)))
    parts = max(1, side // block)
    return Workload("disks_%d_%d" % (k, n), n, n, k0, (pml,) * 4, 3, 1e-8, parts, parts, overlap,
                    local_pml, 3, 1e-8, cells, np.stack(bs), meta=dict(seed=seed0 + k, lam=lam,
                                                                     side=side, rhs=kinds))


def disks_batch(count=48, **kw):
    """The batched workload: problems 0 .. count-1 of disks_problem."""
    return [disks_problem(k, **kw) for k in range(count)]


def waveguides(interior=4096, pml=16, h_nm=20.0, lam_um=1.55, parts=16, overlap=8, local_pml=16,
               seed=4, n_routes=8, n_splits=4, width_um=0.45, eps_si=12.09, eps_sio2=2.085,
               r_min_um=5.0, src_from_pml_um=2.0, subcols=16):
    """Silicon photonic layout (default 4096^2 interior + 16-cell PML = 4128^2
    nodes, h = 20 nm, lambda = 1.55 um = 77.5 cells, 16 x 16 subdomains):
    `n_routes` seeded waveguides (0.45 um Si, eps 12.09, in SiO2, eps 2.085)
    crossing from left to right, each in its own horizontal band, with random
    raised-cosine S-bends of radius >= 5 um; `n_splits` of them split into two
    branches (Y-splits).  Source: the fundamental mode of route 0's cross-section
    (tridiagonal eigen-solve) on the node column 2 um right of the left PML."""
    from . import photonics
    rng = np.random.default_rng(seed)
    n = interior + 2 * pml
    cell_nm = h_nm
    lam = lam_um * 1000.0 / cell_nm
    width = width_um * 1000.0 / cell_nm
    r_min = r_min_um * 1000.0 / cell_nm
    k0 = 2 * math.pi / lam
    band = interior / n_routes
    split_ids = set(rng.choice(n_routes, size=min(n_splits, n_routes), replace=False).tolist())
    paths, starts = [], []
    for i in range(n_routes):
        lo, hi = pml + i * band, pml + (i + 1) * band
        y0 = 0.5 * (lo + hi) + rng.uniform(-0.1, 0.1) * band
        margin = 0.5 * width + 0.1 * band
        if i in split_ids:
            # the trunk stays near the band centre; the branches leave it by +-dy
            half_dy = 0.22 * band
            trunk = photonics.route(-1.0, n, y0, y0 - 0.05 * band, y0 + 0.05 * band, r_min, rng,
                                    n_bends=2, max_dy=0.05 * band)
            xs = float(rng.uniform(0.35, 0.6) * n)
            paths += photonics.y_split(trunk, xs, half_dy, r_min, n)
        else:
            paths.append(photonics.route(-1.0, n, y0, lo + margin, hi - margin, r_min, rng,
                                         n_bends=3, max_dy=0.3 * band))
        starts.append(y0)
    cells = photonics.strip_cells(n, n, paths, width, eps_si, eps_sio2, subcols=subcols)
    col = pml + int(round(src_from_pml_um * 1000.0 / cell_nm))
    # route 0's cross-section window at the source column (its own band)
    nodes = photonics.strip_nodes(n, n, paths[:2] if 0 in split_ids else paths[:1], width, eps_si,
                                  eps_sio2)
    lo, hi = pml, int(pml + band)
    beta2, phi = photonics.fundamental_mode(nodes[lo:hi, col], k0)
    b = np.zeros((n, n), dtype=np.complex128)
    b[lo:hi, col] = phi
    return Workload("waveguides_%d" % n, n, n, k0, (pml,) * 4, 3, 1e-8, parts, parts, overlap,
                    local_pml, 3, 1e-8, cells, b[None],
                    meta=dict(seed=seed, lam=lam, width=width, splits=sorted(split_ids),
                              source_col=col, beta2=beta2, neff=math.sqrt(beta2) / k0))
