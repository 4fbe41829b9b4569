"""Closed-form reference: plane-wave scattering by a dielectric cylinder (Mie series).

TEST INFRASTRUCTURE ONLY (see oracle/fdfd.py).

The paper validates its solver against the analytical series for a dielectric
cylinder under TM incidence (Sec. 3.1, citing Kong's textbook).  Convention
exp(+j w t), incident E_z = exp(-j k0 x) = sum_n j^-n J_n(k0 r) e^{j n phi}
(Jacobi-Anger), k1 = k0 sqrt(eps):
  outside r > a:  E_s = sum_n a_n j^-n H2_n(k0 r) e^{j n phi}
  inside  r < a:  E   = sum_n b_n j^-n J_n(k1 r) e^{j n phi}
Continuity of E_z and dE_z/dr at r = a gives
  a_n = [k1 J_n(k0a) J'_n(k1a) - k0 J'_n(k0a) J_n(k1a)]
        / [k0 H2'_n(k0a) J_n(k1a) - k1 H2_n(k0a) J'_n(k1a)],
  b_n = [J_n(k0a) + a_n H2_n(k0a)] / J_n(k1a).
Bessel and Hankel functions are SciPy's library routines.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def coefficients(k0, a, eps, nmax=None):
    k1 = k0 * np.sqrt(complex(eps))
    if nmax is None:
        x = abs(k1) * a
        nmax = int(math.ceil(x + 4.0 * x ** (1.0 / 3.0))) + 10
    n = np.arange(-nmax, nmax + 1)
    J0, dJ0 = special.jv(n, k0 * a), special.jvp(n, k0 * a)
    J1, dJ1 = special.jv(n, k1 * a), special.jvp(n, k1 * a)
    H0, dH0 = special.hankel2(n, k0 * a), special.h2vp(n, k0 * a)
    an = (k1 * J0 * dJ1 - k0 * dJ0 * J1) / (k0 * dH0 * J1 - k1 * H0 * dJ1)
    bn = (J0 + an * H0) / J1
    return n, an, bn, k1


def scattered_field(k0, a, eps, x, y, nmax=None):
    """E - E_inc at points (x, y) measured from the cylinder axis:
    the scattered field outside, total minus incident inside."""
    n, an, bn, k1 = coefficients(k0, a, eps, nmax)
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    out = np.zeros(r.shape, dtype=np.complex128)
    inside = r < a
    jn = (1j) ** (-n)
    for idx, nn in enumerate(n):
        ph = np.exp(1j * nn * phi)
        ro = r[~inside]
        out[~inside] += an[idx] * jn[idx] * special.hankel2(nn, k0 * ro) * ph[~inside]
        ri = r[inside]
        out[inside] += jn[idx] * (bn[idx] * special.jv(nn, k1 * ri) - special.jv(nn, k0 * ri)) * ph[inside]
    return out
