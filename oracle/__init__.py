"""FP64 CPU oracle for the overlapping-PML source-transfer FDFD solver.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
benchmark's cpu_baseline leg may import it; the HIP library and its Python
binding never do.  Written from the paper (arXiv 2509.20801) in plain
NumPy/SciPy complex128; it shares no code with the GPU path.

Parity status of each function (pins live in tests/test_oracle_*.py):
  fdfd.axis_stretch / assemble   pinned: closed-form eigenpairs, reciprocity,
                                 1D discrete Green's function, Mie series
  fdfd.solve_direct / solve_dense pinned: against each other and residuals
  ddm.partition / local_matrix / SourceTransfer   pinned: N=1 gives A^-1,
                                 residual-support invariant, convergence of
                                 the stationary iteration to the direct solve
  pool.PooledSourceTransfer      the round of SourceTransfer with the factors in
                                 worker processes; pinned: equals SourceTransfer
                                 (complex128 factors) to roundoff
  krylov.fgmres                  pinned: identity preconditioner vs SciPy's
                                 GMRES, Arnoldi relation, exact preconditioner
                                 converges in one step
  ntff.far_field / rcs           pinned: the sampled field of a line source gives
                                 its closed-form far field (second order in h);
                                 vacuum scatters nothing; FDFD cylinder RCS vs the
                                 Mie series (ntff.mie_rcs) at 20 and 40 points per
                                 wavelength, error falling at second order
  mie                            pinned: Jacobi-Anger series of the incident
                                 wave, boundary continuity, eps = 1 gives zero
  nn (learned warm start)        pinned: truncated DFTs vs numpy.fft, every
                                 gradient block vs central differences, GELU
                                 identities, Adam first step, blending is a
                                 partition of unity.  The quality of a trained
                                 network's guess is parity unpinned (no reference
                                 exists); the FP64 true residual judges it.
"""
from . import fdfd, ddm, krylov, mie, nn, ntff, pool  # noqa: F401
