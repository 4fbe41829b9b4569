"""The source-transfer round of oracle.ddm.SourceTransfer with the subdomain
factorisations spread over host worker processes.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The arithmetic is that of
SourceTransfer (same partition, local operators, restriction R_k^I and
full-field prolongation P_k of Eq. (21)); only where the SuperLU factors live
changes: worker w factors and keeps the subdomains k = w, w + W, w + 2W, ...
and answers local-solve requests.  Optionally the factors are kept in
complex64 (SuperLU's single-precision complex LU) to halve their memory: the
round is then an inexact preconditioner, which the flexible GMRES of
oracle.krylov absorbs; the answer is still fixed by the FP64 operator through
the FP64 true residual.

The workers are forked: create the object before the process starts threads
or touches a GPU.
"""
from __future__ import annotations

import multiprocessing as mp

import numpy as np

from . import ddm, fdfd


def _worker(conn, p, eps_cells, ks, dtype):
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)
    subs = ddm.partition(p)
    gax = fdfd.global_axes(p)
    lu = {}
    for k in ks:
        Ak = ddm.local_matrix(p, eps_cells, subs[k], gax).tocsc()
        lu[k] = spla.splu(Ak.astype(dtype))
    conn.send(len(ks))
    while True:
        msg = conn.recv()
        if msg is None:
            conn.close()
            return
        conn.send([(k, lu[k].solve(r.astype(dtype))) for k, r in msg])


class PooledSourceTransfer:
    """z = sum_k P_k A_k^{-1} R_k^I v with the factors held by `workers` processes."""

    def __init__(self, p, eps_cells, workers, factor_dtype=np.complex128):
        self.p = p
        self.nx, self.ny = p["nx"], p["ny"]
        self.subs = ddm.partition(p)
        n = len(self.subs)
        workers = max(1, min(int(workers), n))
        self.groups = [list(range(i, n, workers)) for i in range(workers)]
        ctx = mp.get_context("fork")
        self.conns, self.procs = [], []
        eps = np.asarray(eps_cells)
        for g in self.groups:
            a, b = ctx.Pipe()
            pr = ctx.Process(target=_worker, args=(b, p, eps, g, factor_dtype), daemon=True)
            pr.start()
            self.conns.append(a)
            self.procs.append(pr)
        for c in self.conns:            # every worker has factored its group
            c.recv()

    def _restrict(self, V, s):
        r = np.zeros((s.oy[1] - s.oy[0], s.ox[1] - s.ox[0]), dtype=np.complex128)
        r[s.iy[0] - s.oy[0]:s.iy[1] - s.oy[0], s.ix[0] - s.ox[0]:s.ix[1] - s.ox[0]] = \
            V[s.iy[0]:s.iy[1], s.ix[0]:s.ix[1]]
        return r.ravel()

    def apply(self, v):
        """The round (Eq. (21): the full local fields are summed)."""
        V = np.asarray(v).reshape(self.ny, self.nx)
        for c, g in zip(self.conns, self.groups):
            c.send([(k, self._restrict(V, self.subs[k])) for k in g])
        z = np.zeros((self.ny, self.nx), dtype=np.complex128)
        for c in self.conns:
            for k, u in c.recv():
                s = self.subs[k]
                z[s.oy[0]:s.oy[1], s.ox[0]:s.ox[1]] += np.asarray(u, dtype=np.complex128).reshape(
                    s.oy[1] - s.oy[0], s.ox[1] - s.ox[0])
        return z.ravel()

    def close(self):
        for c in self.conns:
            try:
                c.send(None)
            except (BrokenPipeError, OSError):
                pass
        for pr in self.procs:
            pr.join(timeout=10)
            if pr.is_alive():
                pr.terminate()
        self.conns, self.procs = [], []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
