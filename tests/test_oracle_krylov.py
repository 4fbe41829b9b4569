"""Pins for the oracle's FGMRES against SciPy's GMRES and Arnoldi invariants.  CPU only."""
import numpy as np
import scipy.sparse.linalg as spla

import workloads
from oracle import ddm, fdfd, krylov


def _problem(seed=0):
    w = workloads.configs.small_random(nx=30, ny=26, pml=5, px=2, py=2, overlap=2, local_pml=5,
                                       seed=seed)
    p = w.params()
    return w, p, fdfd.global_matrix(p, w.eps_cells), w.b[0].ravel()


def test_identity_preconditioner_equals_scipy_gmres():
    """One cycle of k steps without preconditioning is the GMRES minimiser over
    the Krylov space K_k(A, b); SciPy's GMRES with restart k and one cycle
    returns the same vector."""
    w, p, A, b = _problem()
    for k in (5, 12):
        x, info = krylov.fgmres(lambda v: A @ v, b, None, tol=1e-30, restart=k, max_iter=k)
        xs, _ = spla.gmres(A, b, rtol=1e-30, atol=0.0, restart=k, maxiter=1)
        assert fdfd.rel_l2(x, xs) < 1e-9


def test_arnoldi_relation_and_orthonormality():
    """A Z_k = V_{k+1} H_k and V^H V = I for the flexible variant."""
    w, p, A, b = _problem(1)
    B = ddm.SourceTransfer(p, w.eps_cells)
    x, info = krylov.fgmres(lambda v: A @ v, b, B.apply, tol=1e-30, restart=6, max_iter=6)
    V, Z, H = info["V"], info["Z"], info["H"]
    AZ = np.stack([A @ z for z in Z])
    assert np.linalg.norm(AZ - H.T @ V) <= 1e-12 * np.linalg.norm(AZ)
    # Modified Gram-Schmidt loses orthogonality in proportion to the
    # condition of the Krylov basis; the basis here converges fast.
    assert np.abs(V.conj() @ V.T - np.eye(V.shape[0])).max() < 1e-10


def test_exact_preconditioner_converges_in_one_step():
    w, p, A, b = _problem(2)
    lu = spla.splu(A.tocsc())
    x, info = krylov.fgmres(lambda v: A @ v, b, lu.solve, tol=1e-12, restart=10)
    assert info["iters"] == 1 and info["relres_true"] < 1e-12


def test_residual_estimate_tracks_true_residual():
    w, p, A, b = _problem(3)
    B = ddm.SourceTransfer(p, w.eps_cells)
    x, info = krylov.fgmres(lambda v: A @ v, b, B.apply, tol=1e-10, restart=30)
    assert info["converged"]
    assert abs(info["history"][-1] - info["relres_true"]) < 1e-11


def test_givens_zeroes_second_entry():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a, bb = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s, r = krylov.givens(a, bb)
        G = np.array([[c, s], [-np.conj(s), c]])
        out = G @ np.array([a, bb])
        assert abs(out[1]) < 1e-14 and abs(out[0] - r) < 1e-14
        assert np.allclose(G.conj().T @ G, np.eye(2))
