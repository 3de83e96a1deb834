"""CPU float64 oracle for the closed-shell CCSD PNK solver.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package. It shares no code with
the HIP path.
"""
