"""CPU reference ("oracle") for the Biot parallel-in-time solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package; only the test suite, the smoke check and the CPU-baseline leg of the
benchmark do.  It is a plain, slow, FP64 implementation written directly from the
paper (stabilized P1-P1 finite elements for the two-field quasi-static Biot model,
Sec. 2; backward Euler, eq. (diseq1); the block system eq. (fullysystem)) and
shares no code with the HIP path: it has its own assembly, its own sparse direct
solve and its own statement of the preconditioned inverted iteration.

Modules
  fem         element matrices and global assembly of A, B, C_K, C_beta, loads
  sequential  sequential backward Euler with a scaled sparse LU + refinement
  inverted    the inverted time-stepping sweep (Alg. 2 / Alg. 3) for a given
              preconditioner, in Gauss-Seidel-in-time and Jacobi-in-time order
  precond     the block preconditioners P1 / P2 (Sec. 3.1) with exact or
              multigrid approximations of the A and S_p solves
  gmg         geometric multigrid hierarchy on the nested structured meshes
  analytic    Terzaghi consolidation series and the trigonometric manufactured
              solution of Sec. 4.1
"""
