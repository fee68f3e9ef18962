"""Plain, slow FP64 CPU oracle for the DD-alpha-AMG twisted-mass hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it and shares no code with it.

Every routine follows the textbook definition or the algorithm's steps in the
order the paper (Bacchio et al., "DDalphaAMG for Twisted Mass Fermions",
PoS LATTICE2016) states them, in complex128, with numpy primitives only.

Modules
  dirac        gamma basis, clover term, D_W, D(mu) = D_W + i mu Gamma5     (Sec. 1, Sec. 2)
  stencil      generic nearest-neighbour block stencil (fine and coarse levels)
  sap          Schwarz alternating procedure with block-local MR             (Sec. 1)
  aggregation  Gamma5-compatible aggregation P, P^dagger                     (Sec. 1)
  coarse       Galerkin coarse operator D_c = P^dagger D P + i mu Gamma5,c   (Sec. 1, Eq. 1)
  krylov       MR, GMRES, FGMRES                                             (Sec. 1)
  mg           V-cycle (Eq. 1), adaptive setup, the preconditioned solve
  net          gauge-covariant parallel-transport network (learned setup)

Parity status per function is listed in the module headers; everything that
is not pinned by a test against an outside truth says "parity unpinned".
"""
