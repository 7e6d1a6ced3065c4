"""MI355X-native preconditioned parallel-in-time solver for the two-field Biot model.

The solver itself is the HIP library libbiot_pint.so (C ABI in include/biot_pint.h);
`solver.BiotSolver` is its Python front end and `workloads` holds the seeded
synthetic inputs.
"""
__all__ = ["workloads", "solver", "build"]
