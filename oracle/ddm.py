"""FP64 CPU oracle: overlapping PML-terminated subdomains and the source-transfer round.

TEST INFRASTRUCTURE ONLY (see oracle/fdfd.py).

Follows Sec. 2.3 (Figs. 2-3, Eqs. (14)-(21), Algorithm 1) with these readings:
  * Partition (Fig. 3): the node grid, global PML included, is cut into
    px x py non-overlapping boxes I_k; the physical interior is split as evenly
    as possible and each edge box also takes the global PML on its side.
  * Each box is extended on every side that faces a neighbour by
    e = overlap + local_pml nodes: `overlap` unstretched cells and then a local
    PML of `local_pml` cells with the grading of Eqs. (11)-(13); the local PML's
    interface half point lies `overlap` cells beyond the edge of I_k.  Sides on
    the global boundary keep the global stretch.  The result is Omega_k.
  * Local operator A_k: the same five-point SC-PML stencil on Omega_k with the
    local stretch arrays, the global node permittivity, Dirichlet outside.
  * One source-transfer round is z = B v = sum_k P_k A_k^{-1} R_k^I v, where
    R_k^I keeps v on I_k and zeroes the extension, and P_k adds the FULL local
    field, extension included, into the global vector (Eq. (21) sums all local
    fields).  Applied to the residual b - A x this is exactly one Jacobi round
    of Algorithm 1: on I_p the residual of the summed field equals the sources
    transferred from the neighbours' overlap fields (Eqs. (16)-(19)).
  * The local systems are solved with SuperLU (a sparse direct LU of the form
    of Eq. (22)-(23)); its result is A_k^{-1} r up to rounding, which is all the
    multifrontal factorisation of the paper defines.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from . import fdfd


@dataclass
class Sub:
    k: int
    kx: int
    ky: int
    ix: tuple   # I_k x range [a, b) in global nodes
    iy: tuple
    ox: tuple   # Omega_k x range [a, b)
    oy: tuple


def split_axis(n, pml_lo, pml_hi, parts):
    """Cut [0, n) into `parts` contiguous ranges: the interior [pml_lo, n-pml_hi)
    is divided as evenly as possible (earlier blocks get the remainder) and the
    first/last block also take the global PML on their side."""
    w = n - pml_lo - pml_hi
    base, rem = divmod(w, parts)
    cuts = [pml_lo]
    for k in range(parts):
        cuts.append(cuts[-1] + base + (1 if k < rem else 0))
    cuts[0] = 0
    cuts[-1] = n
    return [(cuts[k], cuts[k + 1]) for k in range(parts)]


def partition(p):
    e = p["overlap"] + p["local_pml"]
    pxl, pxh, pyl, pyh = p["pml"]
    xr = split_axis(p["nx"], pxl, pxh, p["px"])
    yr = split_axis(p["ny"], pyl, pyh, p["py"])
    subs = []
    for ky in range(p["py"]):
        for kx in range(p["px"]):
            ix, iy = xr[kx], yr[ky]
            ox = (ix[0] - (e if kx > 0 else 0), ix[1] + (e if kx < p["px"] - 1 else 0))
            oy = (iy[0] - (e if ky > 0 else 0), iy[1] + (e if ky < p["py"] - 1 else 0))
            subs.append(Sub(len(subs), kx, ky, ix, iy, ox, oy))
    return subs


def local_axis(g_s, g_sh, o_rng, i_rng, lo_ext, hi_ext, overlap, Lloc, m, R, k0, dlt):
    """Stretch arrays on Omega_k along one axis.

    g_s, g_sh: global arrays (node i, half point i-1/2).  o_rng/i_rng: Omega_k
    and I_k ranges.  On an extended side the local PML has its interface half
    point `overlap` cells beyond I_k's edge; elsewhere the global values apply.
    """
    a, b = o_rng
    n = b - a
    s = g_s[a:b].copy()
    sh = g_sh[a:b + 1].copy()
    if lo_ext:
        iface = i_rng[0] - overlap          # node index just inside the interface
        for u in range(1, Lloc + 1):        # PML node u sits at global node iface - u
            s[iface - u - a] = fdfd.stretch((u - 0.5) * dlt, Lloc, m, R, k0, dlt)
        for u in range(0, Lloc + 1):        # half node u at (iface - u) - 1/2
            sh[iface - u - a] = fdfd.stretch(u * dlt, Lloc, m, R, k0, dlt)
    if hi_ext:
        iface = i_rng[1] + overlap          # first node beyond the physical overlap
        for u in range(1, Lloc + 1):        # PML node u at global node iface - 1 + u
            s[iface - 1 + u - a] = fdfd.stretch((u - 0.5) * dlt, Lloc, m, R, k0, dlt)
        for u in range(0, Lloc + 1):        # half node u at (iface + u) - 1/2
            sh[iface + u - a] = fdfd.stretch(u * dlt, Lloc, m, R, k0, dlt)
    assert len(s) == n
    return s, sh


def local_matrix(p, eps_cells, sub, gaxes=None):
    sx, sxh, sy, syh = gaxes if gaxes is not None else fdfd.global_axes(p)
    lm, lR = p["local_pml_order"], p["local_pml_R"]
    lsx, lsxh = local_axis(sx, sxh, sub.ox, sub.ix, sub.ox[0] < sub.ix[0], sub.ox[1] > sub.ix[1],
                           p["overlap"], p["local_pml"], lm, lR, p["k0"], p["dx"])
    lsy, lsyh = local_axis(sy, syh, sub.oy, sub.iy, sub.oy[0] < sub.iy[0], sub.oy[1] > sub.iy[1],
                           p["overlap"], p["local_pml"], lm, lR, p["k0"], p["dy"])
    cells = np.asarray(eps_cells)[sub.oy[0]:sub.oy[1] + 1, sub.ox[0]:sub.ox[1] + 1]
    return fdfd.assemble(cells, p["k0"], p["dx"], p["dy"], lsx, lsxh, lsy, lsyh)


class SourceTransfer:
    """Factors of every A_k and the round z = B v (Algorithm 1, step 2)."""

    def __init__(self, p, eps_cells):
        self.p = p
        self.nx, self.ny = p["nx"], p["ny"]
        self.subs = partition(p)
        gaxes = fdfd.global_axes(p)
        self.A = [local_matrix(p, eps_cells, s, gaxes) for s in self.subs]
        self.lu = [spla.splu(Ak.tocsc()) for Ak in self.A]

    def restrict(self, v, s):
        """R_k^I v on Omega_k: v on I_k, zero on the extension."""
        V = np.asarray(v).reshape(self.ny, self.nx)
        r = np.zeros((s.oy[1] - s.oy[0], s.ox[1] - s.ox[0]), dtype=np.complex128)
        r[s.iy[0] - s.oy[0]:s.iy[1] - s.oy[0], s.ix[0] - s.ox[0]:s.ix[1] - s.ox[0]] = \
            V[s.iy[0]:s.iy[1], s.ix[0]:s.ix[1]]
        return r.ravel()

    def local_solve(self, k, r):
        return self.lu[k].solve(np.asarray(r, dtype=np.complex128))

    def apply(self, v):
        """z = sum_k P_k A_k^{-1} R_k^I v (Eq. (21) sums the full local fields)."""
        z = np.zeros((self.ny, self.nx), dtype=np.complex128)
        for s in self.subs:
            u = self.local_solve(s.k, self.restrict(v, s))
            z[s.oy[0]:s.oy[1], s.ox[0]:s.ox[1]] += u.reshape(s.oy[1] - s.oy[0], s.ox[1] - s.ox[0])
        return z.ravel()


def overlap_energy(B, v):
    """The round z = B v together with the quantity of Eq. (20): the sum over the
    subdomains of the 2-norm of their local field on the overlapping region,
    i.e. on Omega_k outside I_k (the part E^F that is transferred)."""
    z = np.zeros((B.ny, B.nx), dtype=np.complex128)
    tot = 0.0
    for s in B.subs:
        u = B.local_solve(s.k, B.restrict(v, s)).reshape(s.oy[1] - s.oy[0], s.ox[1] - s.ox[0])
        z[s.oy[0]:s.oy[1], s.ox[0]:s.ox[1]] += u
        mask = np.ones(u.shape, dtype=bool)
        mask[s.iy[0] - s.oy[0]:s.iy[1] - s.oy[0], s.ix[0] - s.ox[0]:s.ix[1] - s.ox[0]] = False
        tot += float(np.linalg.norm(u[mask]))
    return z.ravel(), tot


def stationary_eq20(A, B, b, tol, max_rounds):
    """Algorithm 1 with the stop rule of Eq. (20): rounds continue while the
    overlap energy of the last round is at least tol times that of the initial
    local solves (x_0 = B b).  Returns x, the energies and the relative residuals."""
    x, e0 = overlap_energy(B, b)
    energies = [e0]
    hist = [fdfd.relres(A, x, b)]
    while len(energies) <= max_rounds and not (energies[-1] < tol * e0):
        z, e = overlap_energy(B, b - A @ x)
        x = x + z
        energies.append(e)
        hist.append(fdfd.relres(A, x, b))
    return x, energies, hist


def stationary(A, B, b, rounds):
    """Algorithm 1 as a stationary iteration: x_0 = B b (initial local solves,
    Eq. (14)), then x <- x + B (b - A x) (transferred sources, Eqs. (18)-(19));
    the summed field is Eq. (21).  Returns the iterates' relative residuals."""
    x = B.apply(b)
    hist = [fdfd.relres(A, x, b)]
    for _ in range(rounds):
        x = x + B.apply(b - A @ x)
        hist.append(fdfd.relres(A, x, b))
    return x, hist


# ---------------------------------------------------------------------------
# Multiplicative (sweeping) order of the source transfer.
#
# The paper runs the rounds in parallel over all subdomains (Jacobi).  The
# sweeping source-transfer methods it builds on (Sec. 1: the multiplicative
# and diagonal-sweep forms of Leng et al., Dai et al., Chen and Xiang) visit the
# subdomains in stages instead: each stage solves its subdomains with the
# residual that the stages before it left, so a wave crosses many subdomains in
# one application.  With stages S_1, ..., S_T the application is
#     z = 0;  for each stage t:  z <- z + sum_{k in S_t} P_k A_k^{-1} R_k^I (v - A z),
# the local operators, restriction and full-field prolongation being those of
# the Jacobi round above.  Orders: "rows" (subdomain rows up, then back down),
# "rows_cols" (rows up and down, then columns right and back), "diagonal"
# (anti-diagonals kx + ky rising and falling, then the diagonals
# kx + (py - 1 - ky) rising and falling: four corner-to-corner directions),
# "checker" (two colours: the subdomains with kx + ky even, then those with
# kx + ky odd, so that no stage holds two edge neighbours; the multiplicative
# Schwarz form with the fewest stages).
# ---------------------------------------------------------------------------

ORDERS = ("additive", "rows", "rows_cols", "diagonal", "checker")


def sweep_stages(subs, px, py, order):
    """Stages (lists of subdomain indices) of a sweeping order."""
    if order == "additive":
        return [[s.k for s in subs]]
    rows = [[s.k for s in subs if s.ky == j] for j in range(py)]
    cols = [[s.k for s in subs if s.kx == i] for i in range(px)]
    if order == "rows":
        return rows + rows[-2::-1]
    if order == "rows_cols":
        return rows + rows[-2::-1] + cols + cols[-2::-1]
    if order == "diagonal":
        nd = px + py - 1
        d1 = [[s.k for s in subs if s.kx + s.ky == d] for d in range(nd)]
        d2 = [[s.k for s in subs if s.kx + (py - 1 - s.ky) == d] for d in range(nd)]
        return d1 + d1[-2::-1] + d2 + d2[-2::-1]
    if order == "checker":
        colours = [[s.k for s in subs if (s.kx + s.ky) % 2 == c] for c in (0, 1)]
        return [c for c in colours if c]
    raise ValueError("unknown order %r" % (order,))


def sweep_apply(B, A, v, stages):
    """One application of the staged (multiplicative) source transfer:
    z = 0, then for every stage z += sum_k P_k A_k^{-1} R_k^I (v - A z)."""
    v = np.asarray(v, dtype=np.complex128).ravel()
    z = np.zeros(B.nx * B.ny, dtype=np.complex128)
    for stage in stages:
        r = v - A @ z
        Z = z.reshape(B.ny, B.nx)
        for k in stage:
            s = B.subs[k]
            u = B.local_solve(k, B.restrict(r, s))
            Z[s.oy[0]:s.oy[1], s.ox[0]:s.ox[1]] += u.reshape(s.oy[1] - s.oy[0], s.ox[1] - s.ox[0])
        z = Z.ravel()
    return z
