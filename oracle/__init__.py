"""Plain CPU oracle for the FP64 Jacobi3D sweep -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package; the product path (the HIP library and its binding) never does.
"""
