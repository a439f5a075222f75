"""CPU FP64 oracle for the generalized-Stokes hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product path (the HIP library and its
Python binding) never imports or calls anything here.
"""
