"""FP64 CPU oracle for the staggered-grid direct Poisson solver.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg; the product library never imports it.
"""
