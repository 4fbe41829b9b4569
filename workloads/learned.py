"""Seeded inputs of the learned warm start: initial network weights and the
training tiles.  Holds no solver or network arithmetic.

Flat parameter layout (the order both the FP64 reference and the GPU library
read): P_w (W, cin), P_b (W), then for each layer l: Re R_l (W, W, 2M, M),
Im R_l, W_l (W, W), c_l (W); then Q_w (2, W), Q_b (2).
"""
from __future__ import annotations

import math

import numpy as np

from . import configs, geometry, sources


def param_blocks(width, modes, layers, cin):
    """(entries, std) of each block of the flat parameter vector, in layout order.
    Weights are drawn N(0, std^2) with std = 1/sqrt(fan-in); spectral weights
    with std = 1/W (each output mode sums W inputs); biases start at zero."""
    W, M = width, modes
    b = [(W * cin, 1.0 / math.sqrt(cin)), (W, 0.0)]
    for _ in range(layers):
        b += [(W * W * 2 * M * M, 1.0 / W), (W * W * 2 * M * M, 1.0 / W),
              (W * W, 1.0 / math.sqrt(W)), (W, 0.0)]
    b += [(2 * W, 1.0 / math.sqrt(W)), (2, 0.0)]
    return b


def init_params(width, modes, layers, cin, seed):
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(k) * s for k, s in param_blocks(width, modes, layers, cin)]
    return np.concatenate(parts).astype(np.float64)


def tile_workload(seed, interior=256, pml=20, lam=30.0, n_pillars=16, slot=16, substrate_rows=None,
                  source_row=None, parts=2, overlap=8, local_pml=16, subcells=8):
    """One training tile: a 256 x 256 random metasurface generated as the
    1024 x 1024 one (16 pillars on a substrate, current sheet inside it),
    with its own 20-cell PML, split 2 x 2.  Unless given, the substrate height
    is drawn uniformly in [32, 248] rows and the sheet row uniformly in
    [4, height - 4], so that the tiles of a larger grid that hold the sheet
    (with or without the pillars in view) are in the training distribution."""
    n = interior + 2 * pml
    k0 = 2 * math.pi / lam
    rng = np.random.default_rng([seed, 7919])
    if substrate_rows is None:
        substrate_rows = int(rng.integers(32, min(248, interior - 8) + 1))
    if source_row is None:
        source_row = int(rng.integers(4, substrate_rows - 4 + 1))
    cells = geometry.metasurface(n, n, pml, lam, n_pillars, slot, substrate_rows, 12.25, 2.13, seed,
                                 subcells=subcells)
    b = sources.current_sheet(n, n, pml + source_row)[None]
    return configs.Workload("tile_%d" % seed, n, n, k0, (pml,) * 4, 3, 1e-8, parts, parts, overlap,
                            local_pml, 3, 1e-8, cells, b,
                            meta=dict(seed=seed, lam=lam, substrate_rows=substrate_rows,
                                      source_row=source_row))


def tile_origins(interior, tile=256, stride=128):
    """Origins (in interior coordinates) of the overlapping tiles that cover an
    interior x interior square: a grid of stride `stride`, the last tile flush
    with the far edge."""
    if interior <= tile:
        return [0]
    o = list(range(0, interior - tile + 1, stride))
    if o[-1] != interior - tile:
        o.append(interior - tile)
    return o
