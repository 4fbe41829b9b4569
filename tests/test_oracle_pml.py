"""Pins for the PML stretch (Eqs. (10)-(13)) against the discrete 1D Green's
function and placement properties.  CPU only."""
import math

import numpy as np
import pytest

from oracle import fdfd


def _green_1d(n, L, lam, i0, flip=False, m=3, R=1e-8):
    k0, dy = 2 * math.pi / lam, 1e3
    p = dict(nx=n, ny=1, dx=1.0, dy=dy, k0=k0, pml=(L, L, 0, 0), pml_order=m, pml_R=R)
    sx, sxh, sy, syh = fdfd.global_axes(p)
    if flip:
        sx, sxh = sx.conj(), sxh.conj()
    A = fdfd.assemble(np.ones((2, n + 1), complex), k0, 1.0, dy, sx, sxh, sy, syh)
    b = np.zeros(n, complex); b[i0] = 1
    u = fdfd.solve_direct(A, b)
    # One row of Dirichlet-bounded nodes: the y-part is the shift -2/dy^2.
    kap2 = k0 ** 2 - 2 / dy ** 2
    th = math.acos(1 - kap2 / 2)                 # exp(-j th |i - i0|) solves the 3-point equation
    C = 1j / (2 * math.sin(th))                  # jump condition at the source node
    g = C * np.exp(-1j * th * np.abs(np.arange(n) - i0))
    return u, g, C


@pytest.mark.parametrize("lam,L", [(20.0, 16), (12.0, 10), (30.0, 20)])
def test_point_source_matches_outgoing_discrete_green(lam, L):
    """A PML-terminated line reproduces the free-space discrete Green's
    function C exp(-j theta |i-i0|) in the physical region to PML-reflection
    accuracy, and the field decays through the PML."""
    n = 200
    u, g, C = _green_1d(n, L, lam, 100)
    phys = slice(L, n - L)
    assert np.abs(u[phys] - g[phys]).max() <= 1e-4 * abs(C)
    assert abs(u[0]) <= 1e-2 * abs(C) and abs(u[-1]) <= 1e-2 * abs(C)


def test_wrong_sign_pml_fails_green():
    """Control: with the conjugate stretch the PML amplifies and the pin fails."""
    u, g, C = _green_1d(200, 16, 20.0, 100, flip=True)
    assert np.abs(u[16:184] - g[16:184]).max() > 0.5 * abs(C)


def test_stretch_layout():
    """s = 1 on physical nodes and on the interface half points; the loss grows
    monotonically to the outer half point, where sigma/(w eps0) = sigma_max."""
    n, L, m, R, k0 = 40, 8, 3, 1e-8, 0.5
    s, sh = fdfd.axis_stretch(n, L, L, m, R, k0, 1.0)
    assert np.all(s[L:n - L] == 1) and np.all(sh[L:n - L + 1] == 1)
    assert np.all(s.real == 1) and np.all(sh.real == 1)
    im_lo = -np.concatenate([sh[:L + 1][::-1]]).imag     # depth 0 .. L
    assert np.all(np.diff(im_lo) > 0)
    assert math.isclose(-sh[0].imag, abs(fdfd.sigma_hat_max(L, m, R, k0, 1.0)), rel_tol=1e-14)
    # Integer nodes interleave the half nodes in depth.
    for u in range(1, L + 1):
        assert -sh[L - u + 1].imag < -s[L - u].imag < -sh[L - u].imag
    # Mirror symmetry of the two sides.
    assert np.allclose(s, s[::-1]) and np.allclose(sh, sh[::-1])


def test_sigma_max_matches_theoretical_reflection():
    """Eq. (13): the continuous graded PML backed by a wall reflects
    exp(-2 k0 int sigma/(w eps0) drho) = R(0) at normal incidence."""
    for (L, m, R, k0, d) in [(16, 3, 1e-8, 2 * math.pi / 20, 1.0), (8, 2, 1e-6, 1.3, 0.5)]:
        smax = abs(fdfd.sigma_hat_max(L, m, R, k0, d))
        # int_0^{L d} smax (rho/(L d))^m drho = smax L d / (m + 1)
        assert math.isclose(math.exp(-2 * k0 * smax * L * d / (m + 1)), R, rel_tol=1e-12)
