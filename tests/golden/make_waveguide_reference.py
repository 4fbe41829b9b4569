"""Writes tests/golden/waveguides_4128_samples.json: the oracle's solution of the
4128 x 4128 waveguide workload (4096^2 interior + 16-cell PML, h = 20 nm,
lambda = 1.55 um, seed 4, fundamental-mode source of route 0) at 4096 seeded
sample nodes, plus its norm, true residual and iteration count.

A global direct solve does not fit this host (17M DoF), so the oracle solves it
by its own domain decomposition: FGMRES (oracle.krylov, FP64) right-
preconditioned by the source-transfer round of oracle.pool (16 x 16 subdomains,
the SuperLU factors spread over host processes and kept in complex64), run to
FP64 true rel-res <= 1e-13.  The same method is validated first on the
1064 x 1064 metasurface against the oracle's direct solution stored in
metasurface_1064_samples.json (relative error at its samples <= 1e-10).
Calls only oracle/ and the input generators.

Run: python tests/golden/make_waveguide_reference.py [workers]   (tens of minutes, ~35 GB)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import fdfd, krylov, pool  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def ddm_solve(w, workers, tol, restart, label):
    p = w.params()
    t0 = time.time()
    P = pool.PooledSourceTransfer(p, w.eps_cells, workers, np.complex64)   # forks first
    A = fdfd.global_matrix(p, w.eps_cells)
    b = w.b[0].ravel()
    print("%s: factors ready after %.1f s" % (label, time.time() - t0), flush=True)
    calls = [0]

    def matvec(v):
        calls[0] += 1
        if calls[0] % 20 == 0:
            print("%s: %d operator applications, %.1f s" % (label, calls[0], time.time() - t0),
                  flush=True)
        return A @ v

    hist = []
    try:
        x, info = krylov.fgmres(matvec, b, P.apply, tol=tol, restart=restart, max_iter=5000,
                                history=hist)
    finally:
        P.close()
    rr = fdfd.relres(A, x, b)
    print("%s: %d iterations, true rel-res %.3e, %.1f s" % (label, info["iters"], rr,
                                                           time.time() - t0), flush=True)
    return x, rr, info["iters"], time.time() - t0


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    # 1. the method against the direct solution on the metasurface workload
    ref = json.load(open(os.path.join(HERE, "metasurface_1064_samples.json")))
    w2 = workloads.configs.metasurface_sheet()
    x2, rr2, it2, _ = ddm_solve(w2, workers, 1e-13, 20, "metasurface")
    idx = np.asarray(ref["index"])
    xr = np.asarray(ref["re"]) + 1j * np.asarray(ref["im"])
    err = np.linalg.norm(x2[idx] - xr) / np.linalg.norm(xr)
    print("metasurface: DDM vs direct at the samples: %.3e" % err, flush=True)
    if not (err <= 1e-10 and rr2 <= 1e-13):
        raise SystemExit("validation of the DDM oracle against the direct solve failed")
    del x2
    # 2. the waveguide workload
    w = workloads.configs.waveguides()
    x, rr, iters, secs = ddm_solve(w, workers, 1e-13, 20, "waveguides")
    if not rr <= 1e-13:
        raise SystemExit("waveguide solve did not reach rel-res 1e-13")
    rng = np.random.default_rng(20261203)
    core = np.flatnonzero(np.abs(x) > 1e-3 * np.abs(x).max())       # where the field lives
    pick = np.concatenate([rng.choice(x.size, size=2048, replace=False),
                           rng.choice(core, size=2048, replace=False)])
    pick = np.unique(pick)
    out = dict(workload="waveguides(interior=4096, pml=16, h=20 nm, lambda=1.55 um, parts=16, seed=4)",
               solver="oracle.krylov.fgmres (FP64, restart 20) with the oracle.pool round "
                      "(16 x 16 subdomains, complex64 SuperLU factors)",
               validation=dict(metasurface_err_at_samples=err, metasurface_relres=rr2,
                               metasurface_iters=it2),
               relres=rr, iters=iters, norm=float(np.linalg.norm(x)), index=pick.tolist(),
               re=x[pick].real.tolist(), im=x[pick].imag.tolist(), seconds=secs)
    path = os.path.join(HERE, "waveguides_4128_samples.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
