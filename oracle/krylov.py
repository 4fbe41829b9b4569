"""FP64 CPU oracle: right-preconditioned flexible GMRES (Saad 1993).

TEST INFRASTRUCTURE ONLY (see oracle/fdfd.py).

The paper iterates Algorithm 1 as a stationary scheme; the accelerated form
used here wraps one source-transfer round as the (possibly inexact, hence
flexible) right preconditioner.  Plain textbook steps:
  r0 = b - A x0, beta = |r0|, v1 = r0 / beta, g = beta e1;
  for j: z_j = M(v_j); w = A z_j; modified Gram-Schmidt against v_1..v_j gives
  column j of the Hessenberg matrix H; h_{j+1,j} = |w|; v_{j+1} = w / h_{j+1,j};
  complex Givens rotations reduce H to triangular form and |g_{j+1}| is the
  residual norm of the least-squares iterate;
  at the end of a cycle x = x0 + Z y with H y = g and the true residual is
  recomputed; restart while it is above tol*|b|.
"""
from __future__ import annotations

import numpy as np


def givens(a, b):
    """Complex rotation (c real, s complex) with [c, s; -conj(s), c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b)
    na = abs(a)
    nrm = np.hypot(na, abs(b))
    c = na / nrm
    s = (a / na) * np.conj(b) / nrm
    r = (a / na) * nrm
    return c, s, r


def fgmres(matvec, b, precond=None, x0=None, tol=1e-10, restart=30, max_iter=1000,
           history=None):
    """Solve A x = b.  matvec(v) = A v, precond(v) = M v (None = identity).

    Returns (x, info) with info = dict(iters, relres_true, converged, history,
    V, Z, H) where V, Z, H are the last cycle's Arnoldi quantities.
    """
    b = np.asarray(b, dtype=np.complex128).ravel()
    n = b.size
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128).ravel()
    M = precond if precond is not None else (lambda v: v.copy())
    bnorm = np.linalg.norm(b)
    hist = [] if history is None else history
    it = 0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    hist.append(beta / bnorm)
    last = {}
    if beta <= tol * bnorm:
        return x, dict(iters=0, relres_true=beta / bnorm, converged=True, history=hist)
    while it < max_iter:
        V = np.zeros((restart + 1, n), dtype=np.complex128)
        Z = np.zeros((restart, n), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)   # Hessenberg (unrotated)
        Rm = np.zeros((restart + 1, restart), dtype=np.complex128)  # rotated, upper triangular
        cs = np.zeros(restart)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            Z[j] = M(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):                 # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] == 0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            Hr = H[:, j].copy()                    # rotate a copy of column j
            for i in range(j):
                t = cs[i] * Hr[i] + sn[i] * Hr[i + 1]
                Hr[i + 1] = -np.conj(sn[i]) * Hr[i] + cs[i] * Hr[i + 1]
                Hr[i] = t
            c, s, rr = givens(Hr[j], Hr[j + 1])
            cs[j], sn[j] = c, s
            Hr[j], Hr[j + 1] = rr, 0.0
            Rm[:, j] = Hr
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or breakdown or it >= max_iter:
                break
        k = j_done
        y = np.linalg.solve(np.triu(Rm[:k, :k]), g[:k])
        x = x + Z[:k].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        last = dict(V=V[:k + 1], Z=Z[:k], H=H[:k + 1, :k])
        if beta <= tol * bnorm:
            return x, dict(iters=it, relres_true=beta / bnorm, converged=True, history=hist, **last)
    return x, dict(iters=it, relres_true=beta / bnorm, converged=False, history=hist, **last)
