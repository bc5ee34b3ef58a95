"""FP64 CPU oracle for the matrix-free operator and its solvers.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.
"""
