"""Plain FP64 CPU oracle of the support-graph-preconditioned CG solve.

TEST INFRASTRUCTURE ONLY: the GPU library never imports, links or runs
anything from this package.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.
"""
