"""Writes tests/golden/metasurface_1064_samples.json: the oracle's direct FP64
solution of the 1064 x 1064 metasurface workload (1024^2 interior, 20-cell PML,
lambda = 30 cells, seed 2, current sheet) at 4096 seeded sample nodes plus the
global norm.  Calls only oracle/ and the input generators.

Run: python tests/golden/make_metasurface_reference.py   (SuperLU; a few minutes)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import fdfd  # noqa: E402


def main():
    w = workloads.configs.metasurface_sheet()
    p = w.params()
    A = fdfd.global_matrix(p, w.eps_cells)
    b = w.b[0].ravel()
    t0 = time.time()
    x = fdfd.solve_direct(A, b, refine=2)
    rr = fdfd.relres(A, x, b)
    rng = np.random.default_rng(20260101)
    idx = np.sort(rng.choice(x.size, size=4096, replace=False))
    out = dict(workload="metasurface_sheet(interior=1024, pml=20, lam=30, parts=8, seed=2)",
               solver="oracle.fdfd.solve_direct (SuperLU + 2 refinement steps)",
               relres=rr, norm=float(np.linalg.norm(x)), index=idx.tolist(),
               re=x[idx].real.tolist(), im=x[idx].imag.tolist(), seconds=time.time() - t0)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "metasurface_1064_samples.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path, "relres %.2e" % rr, "%.1f s" % out["seconds"])


if __name__ == "__main__":
    main()
